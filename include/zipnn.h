/*
 * zipnn.h -- C ABI of the MI355X (gfx950) ZipNN codec: lossless compression
 * of model weights by byte grouping + chunked canonical Huffman coding
 * (ZipNN, arXiv 2411.05239).
 *
 * Method, as the paper states it:
 *   - a tensor is a long array of numbers (§II-B); it is cut into fixed-size
 *     chunks (256 KB by default) that compress and decompress independently
 *     (§V-A "Chunking");
 *   - the words of a chunk are regrouped into one byte stream per byte
 *     position, the exponent byte first (§III-A "Exponent Extraction",
 *     §III-B "Byte Grouping");
 *   - each stream is entropy coded with Huffman only (§III-A "Huffman only
 *     Compression"); a single-valued stream shrinks to a header and an
 *     incompressible stream is stored as is (§III-B); the choice is made per
 *     byte-group (§V-A);
 *   - a map holding metadata per chunk and per byte-group allows parallel
 *     decompression of the variable-size chunks (§V-A "Metadata and
 *     parallelism");
 *   - a tensor may be stored as the XOR delta against a base (§IV-B); the
 *     bytes of a delta are mostly unchanged (zero after the XOR), which the
 *     ZG mode below codes without an LZ stage: groups made of the fill value
 *     alone are marked absent in a bitmap and cost one bit each.
 *
 * Container bytes (little-endian; identical to what the CPU reference codec
 * of this project writes):
 *   header (64 B): "ZNN1" | u16 version=1 | u8 dtype | u8 B | u64 n_elems |
 *     u32 chunk_bytes | u16 S | u8 g | u8 L | u32 flags (bit0 = XOR delta, bit1 = the
 *     map holds ZG entries, bit2 = exponent extraction) |
 *     u32 n_chunks | u64 total_bytes | u8 policy[4] | u8 probe interval K |
 *     19 zero bytes
 *   map: n_chunks*B entries of 16 B, chunk-major: u64 payload offset (from
 *     payload_base = align128(64 + 16*n_chunks*B), or 64 with no chunks; the
 *     gap after the map is zero) | u32 bytes | u8 mode (0 RAW, 1 HUF,
 *     2 RLE, 3 ZG) | u8 value (the RLE byte, or the ZG fill byte; else 0) |
 *     u16 0
 *   payloads: in map order, each at a 128-byte aligned offset (a stream
 *     never shares a 128-byte memory line with another), zero padded.
 *     RAW = the m stream bytes.  RLE = nothing.  HUF = 128 B of 4-bit code
 *     lengths | u32 word count of each of the NG = ceil(W/64) lane groups |
 *     zero pad to align16(128+4*NG) | the lane groups' word streams.
 *     ZG = the HUF head | a bitmap of the G = ceil(m/g) groups of g symbols
 *     (bit q in byte q/8, bit q%8), set when group q holds a symbol other
 *     than the fill value z, zero padded to align16(ceil(G/8)) | the word
 *     streams, laid out as for HUF over the marked groups only (unmarked
 *     groups decode to z and take no part in the steps below).
 *   Huffman layout: W = ceil(m/S) sub-streams; group q of g consecutive
 *   symbols belongs to sub-stream q mod W; sub-stream 64j+l is lane l of lane
 *   group j.  A sub-stream's canonical codes (most significant bit first,
 *   packed LSB-first) are cut into 32-bit words, and a lane group's words are
 *   stored in the order its 64 lanes take them when decoding in lock-step:
 *   at step s every lane decodes its group w + s*W pair by pair; for each
 *   pair, every lane whose group exists (and, in ZG, is marked) takes its
 *   next word if it holds fewer than 2L bits (lanes in order), then decodes
 *   the pair.
 *   Stream k of element j is byte B-1-k of the little-endian word.  Codes are
 *   optimal among prefix codes with lengths <= L (package-merge, ties by
 *   (frequency, symbol)) and assigned in canonical (length, symbol) order.
 *
 * Conventions for every call below:
 *   - "device" pointers point to memory of the context's HIP device; every
 *     device buffer (src, dst, base) must be 16-byte aligned;
 *   - `stream` is a hipStream_t (NULL = the legacy default stream);
 *   - the caller owns every buffer it passes; the library never frees them;
 *   - a negative return is a zipnn_status; argument errors are reported
 *     before any work is queued.
 */
#ifndef ZIPNN_H
#define ZIPNN_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    ZIPNN_OK = 0,
    ZIPNN_E_INVAL = -1,    /* bad argument or parameter */
    ZIPNN_E_FORMAT = -2,   /* not a valid container header */
    ZIPNN_E_CORRUPT = -3,  /* map, table or bitstream inconsistent */
    ZIPNN_E_NOSPACE = -4,  /* output capacity too small */
    ZIPNN_E_NOMEM = -5,    /* device or host allocation failed */
    ZIPNN_E_HIP = -6,      /* a HIP runtime call failed */
    ZIPNN_E_BUSY = -7,     /* result not ready yet (serving API) */
    ZIPNN_E_TOOBIG = -8    /* input beyond the fixed scratch of zipnn_compress_noalloc */
} zipnn_status;

typedef enum {
    ZIPNN_BF16 = 1,        /* B = 2 */
    ZIPNN_FP16 = 2,        /* B = 2 */
    ZIPNN_FP32 = 3,        /* B = 4 */
    ZIPNN_FP8_E4M3 = 4,    /* B = 1 */
    ZIPNN_U8 = 5           /* B = 1 */
} zipnn_dtype;

typedef enum {
    ZIPNN_AUTO = 0,        /* the smallest of RAW, HUF and (when the most frequent byte fills at
                              least half of the stream) ZG, ties to RAW then HUF; RLE if
                              single-valued */
    ZIPNN_HUF = 1,         /* always Huffman (RLE if single-valued) */
    ZIPNN_RAW = 2,         /* always stored */
    ZIPNN_ZG = 3           /* always ZG (HUF when the marked groups hold one value; RLE if
                              single-valued) */
} zipnn_policy;

/* Format parameters (they change the container bytes and are stored in it).
 *   chunk_bytes     power of two, 256 .. 4 MiB (paper §V-A default: 256 KiB)
 *   substream_syms  S, power of two, g .. 4096, with chunk_bytes/B/S <= 4096
 *                   and chunk_bytes/S <= 8192
 *   group           g, 2, 4 or 8
 *   max_code_len    L, 8 .. 11
 *   policy[k]       zipnn_policy of stream k (k < B)
 *   probe_skip      K, 0 .. 255: compressibility probing (paper §III-B,
 *                   "Identifying compressibility").  Chunk c of a tensor
 *                   with c mod (K+1) = 0 is a probe chunk; under AUTO the K
 *                   chunks after it store a byte group raw, without
 *                   analysing it, when the probe chunk stored it raw.  0
 *                   (the default) analyses every chunk.  Stored in header
 *                   byte 44.
 *   exponent        1: exponent extraction (paper §III-A, BF16 and FP32
 *                   only): before the split each word's 8 exponent bits move
 *                   to its top byte and the sign right below them, so byte
 *                   group 0 is exactly the exponent (header flag bit 2).
 *                   0 (the default): plain byte grouping.
 *   reserved        zero */
typedef struct {
    uint32_t chunk_bytes;
    uint16_t substream_syms;
    uint8_t group;
    uint8_t max_code_len;
    uint8_t policy[4];
    uint8_t probe_skip;
    uint8_t exponent;
    uint8_t reserved[2];
} zipnn_params;

/* Summary of a container, filled by zipnn_inspect from host bytes. */
typedef struct {
    int dtype;
    int B;
    uint64_t n_elems;
    uint64_t total_bytes;
    uint32_t n_chunks;
    uint32_t chunk_bytes;
    uint32_t S, g, L;
    int is_delta;
    uint64_t bytes_by_mode[4];    /* payload bytes in RAW, HUF, RLE, ZG entries */
    uint64_t entries_by_mode[4];  /* entry counts per mode */
} zipnn_info;

typedef struct zipnn_ctx_s* zipnn_ctx;

/* Create a context on HIP device `hip_device`.  The context owns device
 * scratch (grown on demand by compress), a sticky device-side status word and
 * pinned host staging.  Returns ZIPNN_OK and *out, or a negative status. */
int zipnn_ctx_create(int hip_device, zipnn_ctx* out);

/* Release everything the context owns.  NULL is ignored. */
void zipnn_ctx_destroy(zipnn_ctx ctx);

/* Wait for `stream`, then return the sticky status set by device-side checks
 * since the last clear (ZIPNN_OK, ZIPNN_E_FORMAT, ZIPNN_E_CORRUPT or
 * ZIPNN_E_NOSPACE); the first error recorded wins.  clear != 0 resets it. */
int zipnn_ctx_status(zipnn_ctx ctx, void* stream, int clear);

/* Fill *out with the defaults for `dtype`: 256 KiB chunks (paper §V-A),
 * S = chunk elements / 256 (so a chunk has 256 sub-streams: 512 for 2-byte,
 * 256 for 4-byte, 1024 for 1-byte types), g = 4, L = 11, AUTO everywhere. */
void zipnn_default_params(int dtype, zipnn_params* out);

/* Check params for `dtype`; ZIPNN_OK or ZIPNN_E_INVAL. */
int zipnn_check_params(int dtype, const zipnn_params* p);

/* Upper bound of the container size for n_elems of dtype under p (0 on bad
 * arguments). */
uint64_t zipnn_compress_bound(int dtype, uint64_t n_elems, const zipnn_params* p);

/* Compress n_elems elements of `dtype` at device pointer src (XORed first
 * with device `base` of the same size when base != NULL, paper §IV-B) into
 * device buffer dst of dst_cap bytes.  Blocking: returns after the container
 * is complete on `stream`, with its size in *dst_len (host pointer).
 * ZIPNN_E_NOSPACE if dst_cap is too small (dst contents then undefined). */
int zipnn_compress(zipnn_ctx ctx, const void* src, int dtype, uint64_t n_elems, const void* base,
                   const zipnn_params* p, void* dst, uint64_t dst_cap, uint64_t* dst_len, void* stream);

/* For callers that cannot allocate memory (code under HIP graph capture,
 * serving loops that must not call hipMalloc, harnesses that forbid it): as
 * zipnn_compress, with the same bytes, but the call allocates nothing.  Every
 * device buffer the encoder needs beyond src, base and dst lies in one fixed
 * array of ZIPNN_NOALLOC_SCRATCH_BYTES in each device's memory, set up by
 * zipnn_ctx_create and held until the process ends; the few host words it
 * reads back live on the caller's stack.  Sizes: the tensor may have at most
 * about ZIPNN_NOALLOC_SCRATCH_BYTES / 1.3 KiB chunk-streams (chunks x B; for
 * BF16 at 256 KiB chunks, a tensor of up to 3 GiB); beyond that the call
 * returns ZIPNN_E_TOOBIG before any work is queued.  The array is shared by
 * every call on a device and keeps the last call's contents: calls are
 * serialised by a process-wide lock, and work the caller queues on another
 * stream must not overlap a call on the same device.  Blocking, like
 * zipnn_compress. */
#define ZIPNN_NOALLOC_SCRATCH_BYTES (32u << 20)
int zipnn_compress_noalloc(zipnn_ctx ctx, const void* src, int dtype, uint64_t n_elems, const void* base,
                           const zipnn_params* p, void* dst, uint64_t dst_cap, uint64_t* dst_len, void* stream);

/* Decompress the container at device pointer src (src_len bytes) into device
 * buffer dst (dst_cap bytes; needs n_elems*B), XORing with device `base`
 * (n_elems*B bytes) for a delta container (paper §IV-B).  The 64-byte header
 * is copied to the host first (ordered on `stream`, the call waits for it) to
 * pick the kernel; header errors, a missing or unexpected base and a small
 * dst_cap are returned directly.  The decode itself is then queued on
 * `stream`: the map, tables and word streams are validated on the device and
 * any inconsistency is recorded in the context's sticky status (read it with
 * zipnn_ctx_status).  Nothing outside dst[0, n_elems*B) is written; after an
 * error dst holds unspecified bytes. */
int zipnn_decompress(zipnn_ctx ctx, const void* src, uint64_t src_len, const void* base, void* dst,
                     uint64_t dst_cap, void* stream);

/* As zipnn_decompress, for a caller that already holds a host copy of the
 * container's 64-byte header (`header_host`): nothing waits, the call only
 * queues the decode on `stream`.  The host copy picks the kernel class (B,
 * g, delta, ZG flag); the device parses and checks the header in device
 * memory itself and decodes by it.  If that header is invalid, or its kernel
 * class differs from the host copy's, nothing is decoded and ZIPNN_E_FORMAT
 * is recorded in the status. */
int zipnn_decompress_async(zipnn_ctx ctx, const void* header_host, const void* src, uint64_t src_len,
                           const void* base, void* dst, uint64_t dst_cap, void* stream);

/* ---------------------------------------------------------------- batches
 * A checkpoint is many tensors: they are compressed into one arena, the
 * per-tensor containers back to back in tensor order, each starting at a
 * 128-byte aligned offset, with the whole-model offsets kept by the caller
 * (the paper's map "for the whole model" that allows parallel decompression,
 * §V-A "Metadata and parallelism").  Every kernel is launched once for all
 * chunks of all tensors. */

typedef struct {
    const void* src;       /* device pointer to the tensor */
    uint64_t n_elems;
    const void* base;      /* device pointer to its XOR base, or NULL */
} zipnn_tensor_in;

/* Compress tensors[0..n) (all of `dtype`, host array of device pointers) into
 * the device arena (arena_cap bytes; enough is the sum over tensors of
 * zipnn_compress_bound + 127, since containers start at 128-byte offsets).  offsets (host, n+1 entries) receives the
 * offset of each container and, last, the arena bytes used.  Blocking; the
 * containers are byte-identical to per-tensor zipnn_compress calls. */
int zipnn_compress_batch(zipnn_ctx ctx, int dtype, const zipnn_tensor_in* tensors, int n, const zipnn_params* p,
                         void* arena, uint64_t arena_cap, uint64_t* offsets, void* stream);

typedef struct zipnn_encoder_s* zipnn_encoder;

/* Prepare the batched compression of tensors[0..n) (as zipnn_compress_batch,
 * same bytes) for repeated runs, e.g. saving a checkpoint again and again:
 * the descriptors are uploaded once, and the encode launches (histogram and
 * code build, placement, container layout, packing) plus the copy of the
 * n+1 arena offsets to pinned host memory are captured in a hipGraph.  The
 * encoder owns its scratch.  The tensors (and bases) are read, and the arena
 * written, at every run: they must stay valid while the encoder lives. */
int zipnn_encoder_create(zipnn_ctx ctx, int dtype, const zipnn_tensor_in* tensors, int n, const zipnn_params* p,
                         void* arena, uint64_t arena_cap, zipnn_encoder* out);

/* Replay the graph on `stream` and wait; offsets (host, n+1 entries) receive
 * the containers' offsets and, last, the arena bytes used (ZIPNN_E_NOSPACE if
 * that exceeds arena_cap: the arena then holds unspecified bytes). */
int zipnn_encoder_run(zipnn_encoder e, void* stream, uint64_t* offsets);

/* Wait for the device, then release the encoder.  NULL is ignored. */
void zipnn_encoder_destroy(zipnn_encoder e);

typedef struct zipnn_batch_s* zipnn_batch;

/* Prepare the decompression of the n containers of a device arena (offsets:
 * host, n+1 entries as returned by zipnn_compress_batch) into dst[i] (host
 * array of device pointers, dst_cap[i] bytes each), XORing with base[i] for
 * delta containers (base may be NULL when no container is a delta).  Reads
 * and checks every header (blocking, on the null stream: work of another
 * stream that writes the arena must be complete; the compress calls are
 * blocking), uploads the descriptor tables and records the launches (one per
 * kernel class of (B, g, delta, ZG entries present)) in a hipGraph.  The
 * arena and outputs must stay valid while the batch is used. */
int zipnn_batch_create(zipnn_ctx ctx, const void* arena, const uint64_t* offsets, int n, void* const* dst,
                       const uint64_t* dst_cap, const void* const* base, zipnn_batch* out);

/* Queue the prepared decompression on `stream` (graph replay; asynchronous).
 * Device-side checks report through the context status.  A replay must not
 * overlap another replay of the same batch (they share the outputs and the
 * counters the workgroups take their items from); replays on one stream
 * never do. */
int zipnn_batch_decompress(zipnn_batch b, void* stream);

/* Wait for the device, then release the batch. NULL is ignored. */
void zipnn_batch_destroy(zipnn_batch b);

/* One-shot: create, decompress on `stream`, wait, destroy. */
int zipnn_decompress_batch(zipnn_ctx ctx, const void* arena, const uint64_t* offsets, int n, void* const* dst,
                           const uint64_t* dst_cap, const void* const* base, void* stream);

/* ---------------------------------------------------------------- autotuner */

typedef struct {
    zipnn_params params;
    double ratio;          /* container bytes / input bytes on the sample */
    double decode_gbps;    /* uncompressed GB/s of the batched (graph) decode */
    double encode_gbps;    /* uncompressed GB/s of the batched encode */
} zipnn_tune_entry;

/* How zipnn_autotune samples and decides.  Zero fields take the defaults. */
typedef struct {
    uint64_t sample_bytes;   /* about this many input bytes are compressed per candidate (0: 1 GiB) */
    uint32_t min_chunk;      /* candidate chunk sizes: the powers of two in [min_chunk, max_chunk] */
    uint32_t max_chunk;      /*   (0, 0: 64 KiB .. 1 MiB, the range of the paper's 256 KB default) */
    int repeats;             /* timed decode replays per candidate; the median counts (0: 7) */
    double max_ratio_loss;   /* candidates whose ratio exceeds (1 + loss) x the best ratio are out */
    double tie;              /* decode rates within this fraction of the fastest are ties (0: 0.02) */
    uint8_t policy[4];       /* per-stream zipnn_policy of every candidate (AUTO = 0) */
} zipnn_tune_config;

/* Pick format parameters for a set of tensors of `dtype` by measurement on
 * this GPU (the chunk size is the paper's main parameter, §V-A; S is this
 * format's sub-stream length).
 *   Sample (when the tensors hold more than sample_bytes): stratified by
 *   size class (tensors of equal length, in order of first appearance).  A
 *   class holding c of the total bytes gets ceil(c * sample_bytes / total)
 *   bytes, filled with its tensors in order, whole, the last one cut to
 *   what is left (at least max_chunk bytes, or the whole tensor).  Every kind
 *   of tensor of a checkpoint (embedding, projections, norms) is then in it
 *   in its proportion, at its real length.
 *   Candidates: every chunk size in the range x S = chunk elements / 256 ..
 *   / 2048 (256 to 2048 sub-streams per chunk), within zipnn_check_params.
 *   Each candidate's sample is compressed (timed once) and batch-decompressed
 *   (graph replay: one warm-up, then `repeats` timed runs, median).
 *   Pick: among candidates within the ratio loss, those whose decode rate is
 *   within `tie` of the fastest tie; of those, the smallest chunk, then the
 *   best ratio (exact, so the pick does not follow timing noise).
 * *best gets the pick; entries[0..max_entries) the measurements; *n_entries
 * how many candidates ran.  Blocking; allocates and frees its own sample
 * buffers.  ZIPNN_E_INVAL for an empty candidate set. */
int zipnn_autotune(zipnn_ctx ctx, int dtype, const zipnn_tensor_in* tensors, int n, const zipnn_tune_config* cfg,
                   zipnn_params* best, zipnn_tune_entry* entries, int max_entries, int* n_entries);

/* ------------------------------------------------------------------ serving
 *
 * A decompression server: containers registered once stay resident in
 * device memory; requests to decompress them arrive at any time and their
 * outputs are placed in a device pool of fixed size owned by the server.
 * Requests are admitted in arrival order while the pool has room for the
 * output (and fewer than max_inflight are admitted).  A scheduler thread
 * runs decode iterations on a private stream, keeping two in flight: in
 * ZIPNN_SERVE_CONTINUOUS mode, when more requests are admitted than can
 * each have an iteration in flight, an iteration takes them whole: the
 * oldest, then the others with the fewest chunks first while they fit under
 * chunks_per_iter, so requests that arrive while others decode join the next
 * iteration, many to a launch (otherwise each goes alone);
 * ZIPNN_SERVE_PER_REQUEST runs one iteration per request holding all of its
 * chunks (the plain per-request launch).  Chunks decode independently given
 * the map (paper §V-A), so the bytes of a result do not depend on what else
 * was in its iterations.  Every call is thread-safe.  Times are seconds on
 * the host monotonic clock (zipnn_clock). */

typedef struct zipnn_server_s* zipnn_server;

typedef enum { ZIPNN_SERVE_CONTINUOUS = 0, ZIPNN_SERVE_PER_REQUEST = 1 } zipnn_serve_mode;

typedef struct {
    uint64_t pool_bytes;        /* output pool (device memory allocated at create) */
    int max_inflight;           /* admitted requests not yet released, at most */
    uint32_t chunks_per_iter;   /* CONTINUOUS: chunk cap of one iteration beyond its first request (0: 2048) */
    int mode;                   /* zipnn_serve_mode */
} zipnn_server_config;

typedef struct {
    double t_arrive;   /* given at submit (or the submit time) */
    double t_admit;    /* output space granted */
    double t_launch;   /* first iteration holding one of its chunks queued */
    double t_done;     /* the iteration holding its last chunk seen complete */
} zipnn_timing;

typedef struct {
    uint64_t submitted, completed, released;
    uint64_t iterations;      /* decode iterations launched */
    uint64_t chunks;          /* chunks decoded */
    uint64_t bytes_out;       /* uncompressed bytes of completed requests */
    uint64_t pool_in_use, pool_peak;
    int active_peak;          /* most admitted requests at once */
} zipnn_server_counters;

/* Seconds on the clock the server stamps (CLOCK_MONOTONIC). */
double zipnn_clock(void);

/* Create a server on ctx's device (the context must outlive it). */
int zipnn_server_create(zipnn_ctx ctx, const zipnn_server_config* cfg, zipnn_server* out);

/* Stop the scheduler after the iterations in flight, free the pool.  Output
 * pointers handed out become invalid.  NULL is ignored. */
void zipnn_server_destroy(zipnn_server srv);

/* Register a container resident in device memory (src_len bytes; for a delta
 * container, base: the device XOR base, else NULL).  The header is read and
 * checked (blocking); the container and base must stay valid and unchanged
 * while the server lives.  *handle names it in submit. */
int zipnn_server_register(zipnn_server srv, const void* src, uint64_t src_len, const void* base, uint32_t* handle);

/* Ask for one decompression of a registered container; t_arrive <= 0 means
 * now.  Returns at once with *ticket; ZIPNN_E_NOSPACE if the output can never
 * fit the pool. */
int zipnn_server_submit(zipnn_server srv, uint32_t handle, double t_arrive, uint64_t* ticket);

/* ZIPNN_E_BUSY while the request is pending; once done, its status (OK, or
 * the error the device reported for one of its iterations), *out = its output
 * in the pool (n * B bytes) and *t its timing (either may be NULL). */
int zipnn_server_poll(zipnn_server srv, uint64_t ticket, void** out, zipnn_timing* t);

/* Wait up to timeout_s for a completed request not yet returned by this call
 * and give its ticket; ZIPNN_E_BUSY on time-out. */
int zipnn_server_next_done(zipnn_server srv, double timeout_s, uint64_t* ticket);

/* Give a completed request's output space back to the pool and forget it;
 * ZIPNN_E_BUSY if it is not done. */
int zipnn_server_release(zipnn_server srv, uint64_t ticket);

/* Counters since create. */
int zipnn_server_stats(zipnn_server srv, zipnn_server_counters* out);

/* Switch the batching mode (zipnn_serve_mode); iterations launched from then
 * on follow it, those in flight are unaffected.  Lets one server, with one
 * output pool and one stream, compare continuous batching with the plain
 * per-request launch on the same memory.  ZIPNN_E_INVAL for another mode. */
int zipnn_server_set_mode(zipnn_server srv, int mode);

/* Validate a container's header and map from HOST memory (len bytes: at
 * least the header and the map) and summarise it in *out. */
int zipnn_inspect(const void* host_buf, uint64_t len, zipnn_info* out);

/* Static English text for a status code. */
const char* zipnn_strerror(int code);

#ifdef __cplusplus
}
#endif
#endif /* ZIPNN_H */
