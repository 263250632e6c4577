// Internal declarations shared by the HIP kernels and the host runtime of the
// gfx950 ZipNN codec.  The container layout is documented in include/zipnn.h.
#pragma once

#include <hip/hip_runtime.h>
#include <mutex>
#include <stdint.h>

#include "zipnn.h"

namespace zipnn {

constexpr uint32_t kMinChunk = 256;
constexpr uint32_t kMaxChunk = 4u << 20;
constexpr uint32_t kMaxS = 4096;
constexpr uint32_t kMinG = 2;
constexpr uint32_t kMaxG = 8;
constexpr uint32_t kLanes = 64;             // sub-streams per lane group (one wave)
constexpr uint32_t kMinL = 8;
constexpr uint32_t kMaxL = 11;
constexpr uint32_t kMaxW = 4096;           // sub-streams per chunk and stream
constexpr uint32_t kMaxBW = 8192;          // sub-streams per chunk over all B streams
constexpr uint32_t kLutSize = 1u << kMaxL;  // decode table entries per stream
constexpr uint32_t kFlagDelta = 1;
constexpr uint32_t kFlagZg = 2;               // the map holds ZG entries
constexpr uint32_t kFlagExp = 4;              // exponent extraction (BF16 / FP32)
constexpr int kModeRaw = 0, kModeHuf = 1, kModeRle = 2, kModeZg = 3;
constexpr int kBlock = 256;                 // threads per workgroup (4 waves)

__host__ __device__ inline uint64_t align16(uint64_t v) { return (v + 15u) & ~uint64_t(15); }

// Allocations that clear the thread's last HIP error when they fail: the
// caller reports the failure, and a later kernel launch checked with
// hipGetLastError must not read it as its own.
inline hipError_t dev_malloc(void** p, size_t n)
{
    const hipError_t e = hipMalloc(p, n);
    if (e != hipSuccess) {
        *p = nullptr;
        (void)hipGetLastError();
    }
    return e;
}
inline hipError_t host_malloc(void** p, size_t n)
{
    const hipError_t e = hipHostMalloc(p, n, hipHostMallocDefault);
    if (e != hipSuccess) {
        *p = nullptr;
        (void)hipGetLastError();
    }
    return e;
}

// Payloads start at multiples of kPayAlign bytes from the container start (and
// containers at such offsets in a batch arena), so that two streams never
// share a 128-byte memory line.
constexpr uint64_t kPayAlign = 128;
__host__ __device__ inline uint64_t align_pay(uint64_t v) { return (v + kPayAlign - 1) & ~(kPayAlign - 1); }
// Offset of the payload area: header + map, aligned (64 with no chunks).
__host__ __device__ inline uint64_t payload_base_of(uint64_t n_chunks, uint64_t B)
{
    return n_chunks ? align_pay(64 + 16 * n_chunks * B) : 64;
}
__host__ __device__ inline bool pow2(uint64_t v) { return v && !(v & (v - 1)); }

__host__ __device__ inline int dtype_bytes(int dt)
{
    return dt == ZIPNN_BF16 || dt == ZIPNN_FP16 ? 2 : dt == ZIPNN_FP32 ? 4 : dt == ZIPNN_FP8_E4M3 || dt == ZIPNN_U8 ? 1 : 0;
}

__host__ __device__ inline int check_params(int B, uint32_t chunk, uint32_t S, uint32_t g, uint32_t L)
{
    if (!B || !pow2(chunk) || chunk < kMinChunk || chunk > kMaxChunk) return ZIPNN_E_INVAL;
    if (!pow2(g) || g < kMinG || g > kMaxG || !pow2(S) || S < g || S > kMaxS) return ZIPNN_E_INVAL;
    if (L < kMinL || L > kMaxL) return ZIPNN_E_INVAL;
    if (chunk / uint32_t(B) / S > kMaxW || chunk / S > kMaxBW) return ZIPNN_E_INVAL;
    return ZIPNN_OK;
}

// Size of the part of a HUF payload that precedes its words: the nibble
// table and one u32 word count per lane group, padded to 16 bytes.
__host__ __device__ inline uint32_t huf_head(uint32_t W)
{
    return uint32_t(align16(128u + 4u * ((W + kLanes - 1) / kLanes)));
}

// Size of the group bitmap of a ZG payload (after the head): one bit per
// group of g symbols, padded to 16 bytes.
__host__ __device__ inline uint32_t zg_bitmap(uint32_t m, uint32_t g)
{
    return uint32_t(align16(((m + g - 1) / g + 7) / 8));
}

// Exponent extraction (paper §III-A) on a register of little-endian words:
// BF16 (B = 2, two words) or FP32 (B = 4).  Forward: sign | exponent |
// fraction becomes exponent | sign | fraction, so the top byte of a word is
// its exponent; the fraction bits stay.  exp_inv undoes it.  Other widths
// pass through.
template <int B>
__host__ __device__ inline uint32_t exp_fwd(uint32_t x)
{
    if constexpr (B == 2) return ((x << 1) & 0xFF00FF00u) | ((x >> 8) & 0x00800080u) | (x & 0x007F007Fu);
    else if constexpr (B == 4) return ((x << 1) & 0xFF000000u) | ((x >> 8) & 0x00800000u) | (x & 0x007FFFFFu);
    else return x;
}
template <int B>
__host__ __device__ inline uint32_t exp_inv(uint32_t x)
{
    if constexpr (B == 2) return ((x >> 1) & 0x7F807F80u) | ((x << 8) & 0x80008000u) | (x & 0x007F007Fu);
    else if constexpr (B == 4) return ((x >> 1) & 0x7F800000u) | ((x << 8) & 0x80000000u) | (x & 0x007FFFFFu);
    else return x;
}

struct Header {
    uint64_t n, total, payload_base;
    uint32_t dtype, B, chunk, S, g, L, flags, n_chunks, E;
};

// Parse and validate a 64-byte header (16-byte aligned words).  Usable on the
// host and on the device.
__host__ __device__ inline int parse_header(const uint32_t* w, uint64_t src_len, Header& h)
{
    if (w[0] != 0x314E4E5Au) return ZIPNN_E_FORMAT;            // "ZNN1"
    if ((w[1] & 0xFFFFu) != 1u) return ZIPNN_E_FORMAT;
    h.dtype = (w[1] >> 16) & 0xFF;
    h.B = w[1] >> 24;
    h.n = uint64_t(w[2]) | (uint64_t(w[3]) << 32);
    h.chunk = w[4];
    h.S = w[5] & 0xFFFF;
    h.g = (w[5] >> 16) & 0xFF;
    h.L = w[5] >> 24;
    h.flags = w[6];
    h.n_chunks = w[7];
    h.total = uint64_t(w[8]) | (uint64_t(w[9]) << 32);
    if (dtype_bytes(int(h.dtype)) != int(h.B) || h.B == 0) return ZIPNN_E_FORMAT;
    if (check_params(int(h.B), h.chunk, h.S, h.g, h.L) != ZIPNN_OK) return ZIPNN_E_FORMAT;
    if (h.flags & ~(kFlagDelta | kFlagZg | kFlagExp)) return ZIPNN_E_FORMAT;
    if ((h.flags & kFlagExp) && h.dtype != ZIPNN_BF16 && h.dtype != ZIPNN_FP32) return ZIPNN_E_FORMAT;
    if (w[11] & ~0xFFu) return ZIPNN_E_FORMAT;   // byte 44 is the probe interval
    for (int i = 12; i < 16; i++)
        if (w[i]) return ZIPNN_E_FORMAT;
    h.E = h.chunk / h.B;
    if ((h.n + h.E - 1) / h.E != h.n_chunks) return ZIPNN_E_FORMAT;
    h.payload_base = payload_base_of(h.n_chunks, h.B);
    if (h.total < h.payload_base || h.total > src_len) return ZIPNN_E_FORMAT;
    return ZIPNN_OK;
}

// One tensor of a (possibly batched) decode.
struct DecDesc {
    const uint8_t* src;
    uint64_t src_len;
    const uint8_t* base;   // XOR base or nullptr
    uint8_t* dst;          // the whole tensor's output (chunk c lands at c * chunk_bytes)
    uint64_t dst_cap;
    uint32_t c_begin;      // chunks [c_begin, min(c_end, n_chunks)) are decoded
    uint32_t c_end;
    int* status;           // where corruption found in its chunks is reported (nullptr: the launch's)
};
constexpr uint32_t kAllChunks = 0xFFFFFFFFu;

// One tensor of a (possibly batched) encode.
struct EncDesc {
    const uint8_t* src;
    const uint8_t* base;
    uint8_t* dst;          // container
    uint64_t dst_cap;
    uint64_t n;
    uint32_t chunk0;       // index of this tensor's first chunk in the scratch arrays
    uint32_t n_chunks;
    uint32_t has_zg;       // set by the placement kernel: some entry is ZG
    uint32_t pad;
};

// Per-(chunk, stream) result of the analysis kernel.
struct EncEntry {
    uint32_t bytes;        // payload bytes
    uint8_t mode;
    uint8_t rle;
    uint16_t pad;
};

// Encode-side code table entry: canonical code | length << 16.
using CodeWord = uint32_t;

struct EncParams {
    uint32_t dtype, B, chunk, S, g, L;
    uint32_t flags;        // kFlagExp; kFlagDelta when some tensor of the launch has an XOR base
    uint32_t skip;         // probe interval K (0: every chunk analysed)
    uint8_t policy[4];
    // Staged packing (nullptr: the exact-size path): every (chunk, stream)
    // owns stage_chunk bytes of `stage` at (global chunk * B + k) *
    // stage_chunk: a ZG bitmap or raw bytes from its start, and lane group j's
    // words at stage_bm + j * stage_lg (StageLayout).
    uint8_t* stage;
    uint32_t stage_chunk, stage_lg, stage_bm;
};

// Staging slots of one launch: a lane of S symbols holds at most S * L code
// bits and takes at most ceil((S L + 2L + 31) / 32) words (the refill rule),
// so a lane group needs at most 64 times that; a chunk of E = chunk / B
// elements has at most ceil(ceil(E / S) / 64) lane groups, and its raw bytes
// (E) fit in that room since L >= 8.
struct StageLayout {
    uint32_t lg, bm, chunk;
};
__host__ __device__ inline StageLayout stage_layout(uint32_t chunk, uint32_t B, uint32_t S, uint32_t g, uint32_t L)
{
    const uint32_t E = chunk / B;
    const uint32_t W = (E + S - 1) / S, NG = (W + kLanes - 1) / kLanes;
    StageLayout st;
    st.lg = uint32_t(align16(uint64_t(kLanes) * 4u * ((S * L + 2u * L + 31u) / 32u + 1u)));
    st.bm = zg_bitmap(E, g);
    const uint64_t c = uint64_t(st.bm) + uint64_t(NG) * st.lg;
    st.chunk = uint32_t(((c > E ? c : uint64_t(E)) + 255u) & ~uint64_t(255));
    return st;
}

// Work items of a decode descriptor: one item per (chunk, slice of kBlock
// sub-streams) over the chunks [c_begin, min(c_end, n_chunks)); the
// tensor's last chunk may have fewer sub-streams than the others.
struct ItemPlan {
    uint32_t slices_full;  // slices per full chunk
    uint32_t slices_last;  // slices of the tensor's last chunk, when the range holds it
    uint32_t c0;           // first chunk of the range
    uint32_t full_chunks;  // chunks of the range with slices_full slices
    uint64_t items;
};

__host__ __device__ inline ItemPlan plan_items(const Header& h, uint32_t c_begin, uint32_t c_end)
{
    ItemPlan p;
    const uint32_t Wf = (h.E + h.S - 1) / h.S;
    p.slices_full = (Wf + kBlock - 1) / kBlock;
    p.slices_last = 0;
    p.c0 = 0;
    p.full_chunks = 0;
    p.items = 0;
    const uint32_t c1 = c_end < h.n_chunks ? c_end : h.n_chunks;
    if (c_begin >= c1) return p;
    p.c0 = c_begin;
    if (c1 < h.n_chunks) {
        p.full_chunks = c1 - c_begin;
    } else {
        p.full_chunks = c1 - 1 - c_begin;
        const uint64_t m_last = h.n - uint64_t(h.n_chunks - 1) * h.E;
        const uint32_t Wl = uint32_t((m_last + h.S - 1) / h.S);
        p.slices_last = (Wl + kBlock - 1) / kBlock;
    }
    p.items = uint64_t(p.full_chunks) * p.slices_full + p.slices_last;
    return p;
}

// Launchers (decode.hip / encode.hip).  A null descriptor array means "the
// single tensor passed by value".
// Decode kernels are specialised on (B, g, delta, zg) taken from the header
// (zg: the header's ZG flag; only those kernels carry the ZG decoder).
struct DecClass {
    uint32_t B, G;
    bool delta, zg;
};
__host__ __device__ inline DecClass dec_class(const Header& h)
{
    return DecClass{h.B, h.g, (h.flags & kFlagDelta) != 0, (h.flags & kFlagZg) != 0};
}
hipError_t launch_decode_one(const Header& h, const DecDesc& one, int* d_status, int grid, hipStream_t s);
// Batched decode: k_plan writes the item prefix (n_desc + 1 entries) and
// zeroes the item counter after it, from which the workgroups take their
// items; d_item_prefix has room for n_desc + 2 entries.
hipError_t launch_decode_batch(const DecClass& k, const DecDesc* d_descs, int n_desc, uint64_t* d_item_prefix,
                               int* d_status, int grid, hipStream_t s);
// Batched decode whose item prefix (plan_items per descriptor) was computed
// on the host and copied beside the descriptors, followed by the item
// counter, zero at launch (n_desc + 2 entries).
hipError_t launch_decode_planned(const DecClass& k, const DecDesc* d_descs, int n_desc, uint64_t* d_item_prefix,
                                 int* d_status, int grid, hipStream_t s);
hipError_t launch_clear_status(int* d_status, hipStream_t s);
hipError_t launch_gather_headers(const uint8_t* arena, const uint64_t* d_offs, int n, void* d_out, hipStream_t s);
int decode_grid_size(int device, const DecClass& k);
// Index of a kernel class in per-class tables (B in {1,2,4}, G in {2,4,8}).
constexpr int kDecClasses = 36;
__host__ __device__ inline int dec_class_index(const DecClass& k)
{
    const int bi = k.B == 1 ? 0 : k.B == 2 ? 1 : 2;
    const int gi = k.G == 2 ? 0 : k.G == 4 ? 1 : 2;
    return ((bi * 3 + gi) * 2 + (k.delta ? 1 : 0)) * 2 + (k.zg ? 1 : 0);
}

// Compress n_desc tensors (descriptors and chunk prefix in device memory)
// into `arena`: analyze -> place -> arena layout (dst of every descriptor,
// headers, arena_off[n_desc+1]) -> pack (maps and payloads).
hipError_t launch_encode(EncDesc* d_descs, int n_desc, const uint32_t* d_chunk_prefix, uint32_t total_chunks,
                         const EncParams& p, uint8_t* arena, uint64_t cap, EncEntry* entries, CodeWord* codes,
                         uint32_t* nwords, uint64_t* offsets, uint64_t* totals, uint64_t* arena_off, hipStream_t s);

hipError_t launch_fill_desc(const EncDesc& one, uint32_t total_chunks, EncDesc* d_desc, uint32_t* d_prefix,
                            hipStream_t s);

// Offsets of the encoder's device scratch for ne = chunks * B entries of n
// tensors (every array 256-byte aligned); `need` is the total.
struct EncScratch {
    size_t entries, codes, offsets, nwords, totals, aoff, descs, prefix, stage, need;
};
// stage_bytes: the staging slots of a staged launch (0: none)
inline EncScratch enc_scratch_layout(size_t ne, size_t n, size_t stage_bytes = 0)
{
    auto a256 = [](size_t v) { return (v + 255) & ~size_t(255); };
    EncScratch L;
    L.entries = 0;
    L.codes = a256(L.entries + ne * sizeof(EncEntry));
    L.offsets = a256(L.codes + ne * 256 * sizeof(CodeWord));
    L.nwords = a256(L.offsets + ne * sizeof(uint64_t));
    L.totals = a256(L.nwords + ne * 64 * sizeof(uint32_t));
    L.aoff = a256(L.totals + n * sizeof(uint64_t));
    L.descs = a256(L.aoff + (n + 1) * sizeof(uint64_t));
    L.prefix = a256(L.descs + n * sizeof(EncDesc));
    L.stage = a256(L.prefix + (n + 1) * sizeof(uint32_t));
    L.need = L.stage + stage_bytes + 256;
    return L;
}

}  // namespace zipnn

// A codec context: the device it runs on, the sticky device-side status and
// the encoder's scratch (grown on demand, serialised by `mu`).
struct zipnn_ctx_s {
    int device = 0;
    int dec_grid[zipnn::kDecClasses] = {};   // persistent decode grid of each kernel class
    int* d_status = nullptr;      // sticky device-side status
    int* h_status = nullptr;      // pinned
    uint64_t* h_total = nullptr;  // pinned, encode sizes
    size_t h_total_cap = 0;
    void* d_scratch = nullptr;    // encode scratch (grown on demand)
    void* fixed_scratch = nullptr;  // the device's fixed scratch array (zipnn_compress_noalloc)
    size_t scratch_cap = 0;
    std::mutex mu;                // serialises users of the scratch
};
