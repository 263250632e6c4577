/*
 * ZipNN oracle (test infrastructure only -- never linked by the product).
 *
 * Container format produced and accepted here (all integers little-endian):
 *
 *   header, 64 bytes:
 *     0  "ZNN1"            4  u16 version = 1     6  u8 dtype     7  u8 B
 *     8  u64 n_elems       16 u32 chunk_bytes     20 u16 S        22 u8 g
 *     23 u8 L              24 u32 flags                           28 u32 n_chunks
 *     32 u64 total_bytes   40 u8 policy[4]        44 u8 probe interval K
 *     45..63 zero
 *   flags: bit0 XOR delta; bit1 the map holds ZG entries (written when it
 *     does; a ZG entry without it is corrupt); bit2 exponent extraction
 *     (BF16 / FP32 only: before the split, each word's exponent moves to its
 *     top 8 bits and the sign right below them); other bits zero.
 *   map at 64: n_chunks*B entries of 16 bytes, chunk-major (entry c*B+k):
 *     u64 offset from payload_base | u32 bytes | u8 mode | u8 value | u16 0
 *     (value: the RLE byte, or the ZG fill byte; zero otherwise)
 *   payload_base = align128(64 + 16*n_chunks*B) (64 when n_chunks = 0);
 *   payloads in map order, each starting at a 128-byte aligned offset;
 *   padding is zero; RLE entries have no bytes and carry the running offset;
 *   total_bytes = payload_base + aligned end.
 *   RAW payload: the m stream bytes.
 *   HUF payload: 128 bytes of 4-bit code lengths (byte i = l[2i] | l[2i+1]<<4)
 *     | u32 word count of each of the NG = ceil(W/64) lane groups | zero pad
 *     to align16(128 + 4*NG) | the word streams of lane groups 0..NG-1.
 *     The coding: W = ceil(m/S) sub-streams; group q of g consecutive symbols
 *     belongs to sub-stream q mod W; a sub-stream's bit string is the
 *     canonical codes of its symbols, most significant bit first, packed
 *     LSB-first (orc_substream_bits).
 *     The layout (the format's choice, made for a decoder that runs 64
 *     sub-streams in lock-step, one per lane of a wavefront): sub-stream
 *     64j+l is lane l of lane group j; each bit string is cut into 32-bit
 *     words; the decode events of a lane group -- (step s, pair p, lane l)
 *     for every pair of symbols of every coded group 64j+l+s*W -- are sorted
 *     by (s, p, l); walking them, a lane holding fewer than 2L bits takes its
 *     next word before its event, and the event's code bits then leave its
 *     buffer.  The words are stored in the order taken (a lane may take one
 *     all-zero word past its last code bit).
 *   ZG payload (fill value z in the map): the HUF head | a bitmap of the
 *     G = ceil(m/g) groups, bit q (byte q/8, bit q%8) set when group q holds
 *     a symbol other than z, zero padded to align16(ceil(G/8)) | the word
 *     streams as for HUF, where only marked groups are coded and give
 *     events; unmarked groups decode to z.
 */
#ifndef ZIPNN_ORACLE_H
#define ZIPNN_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    ORC_OK = 0,
    ORC_E_INVAL = -1,
    ORC_E_FORMAT = -2,
    ORC_E_CORRUPT = -3,
    ORC_E_NOSPACE = -4,
    ORC_E_NOMEM = -5
};
enum { ORC_BF16 = 1, ORC_FP16 = 2, ORC_FP32 = 3, ORC_FP8_E4M3 = 4, ORC_U8 = 5 };
enum { ORC_POLICY_AUTO = 0, ORC_POLICY_HUF = 1, ORC_POLICY_RAW = 2, ORC_POLICY_ZG = 3 };
enum { ORC_MODE_RAW = 0, ORC_MODE_HUF = 1, ORC_MODE_RLE = 2, ORC_MODE_ZG = 3 };
enum { ORC_FLAG_DELTA = 1, ORC_FLAG_ZG = 2, ORC_FLAG_EXP = 4 };

#define ORC_MIN_CHUNK 256u
#define ORC_MAX_CHUNK (4u << 20)
#define ORC_MAX_S 4096u
#define ORC_MIN_G 2u
#define ORC_MAX_G 8u
#define ORC_LANES 64u
#define ORC_MAX_W 4096u
#define ORC_MAX_BW 8192u
#define ORC_MIN_L 8u
#define ORC_MAX_L 11u
#define ORC_PAY_ALIGN 128u   /* payload alignment from the container start */

typedef struct {
    int dtype, B;
    uint64_t n;
    uint32_t chunk_bytes, S, g, L, flags, n_chunks;
    uint64_t total;
    uint8_t policy[4];
    uint32_t skip;
} orc_header;

int orc_check_params(int B, uint32_t chunk_bytes, uint32_t S, uint32_t g, uint32_t L);
void orc_split_stream(const uint8_t* words, uint64_t m, int B, int k, uint8_t* out);
int orc_package_merge(const uint64_t f[256], int L, uint8_t len_out[256]);
void orc_canonical_codes(const uint8_t len[256], int L, uint32_t code[256]);
/* Bit string of sub-stream w of a stream of m symbols (the coding without the
 * word layout): the canonical codes of the symbols of its groups w, w+W, ...
 * (W = ceil(m/S); flags != NULL: only groups with flags[q] != 0), most
 * significant code bit first, packed LSB-first into out (zeroed first). */
int orc_substream_bits(const uint8_t* sym, uint64_t m, uint32_t S, uint32_t g, int L, const uint8_t len[256],
                       const uint8_t* flags, uint64_t w, uint8_t* out, uint64_t out_bytes, uint64_t* nbits);
uint64_t orc_compress_bound(int dtype, uint64_t n, uint32_t chunk_bytes, uint32_t S);
/* skip: probe interval K (0..255).  Chunk c of the tensor is a probe chunk
 * when c mod (K+1) = 0; under AUTO the K chunks after a probe chunk are
 * stored raw without analysis in every byte group the probe stored raw.
 * exp: exponent extraction (BF16 and FP32 only). */
int orc_compress(const void* src, int dtype, uint64_t n, const void* base, uint32_t chunk_bytes, uint32_t S,
                 uint32_t g, uint32_t L, const uint8_t* policy, uint32_t skip, int exp, void* dst, uint64_t dst_cap,
                 uint64_t* dst_len, int nthreads);
int orc_parse_header(const void* src, uint64_t src_len, orc_header* h);
int orc_decompress(const void* src, uint64_t src_len, const void* base, void* dst, uint64_t dst_cap,
                   int nthreads);
int orc_entry(const void* src, uint64_t src_len, uint32_t chunk, int k, uint64_t* off_abs, uint64_t* bytes,
              int* mode, int* rle);

#ifdef __cplusplus
}
#endif
#endif
