// Decode kernels of the gfx950 ZipNN codec.
//
// Work item = (tensor, chunk, slice of up to 256 sub-streams = 4 lane groups).
// Chunks are independent given the map (paper §V-A "Metadata and
// parallelism"); inside a chunk the W sub-streams of every Huffman-coded byte
// group are independent too.  One workgroup (4 waves) takes one item: it
// checks the item's map entries and expands each Huffman table into an LDS
// lookup table shared by its waves; then wave v decodes lane group 4*slice+v
// on its own: lane l owns sub-stream 64*(4*slice+v)+l of EVERY stream of the
// chunk.  All streams of a chunk share (m, S, g), so sub-stream w of every
// stream covers the same elements (groups q = w, w+W, ...): the lane merges
// the B byte groups back into words in registers (the inverse of byte
// grouping, paper §III-A/§III-B), applies the XOR delta (paper §IV-B) and
// writes g whole words with one vector store; a wave writes 64*g*B
// contiguous bytes per group.
//
// A lane group's Huffman words are stored in the order its 64 lanes take them
// when they run in lock-step (step s, pair p: a lane holding fewer than 2L
// bits takes a word, then decodes symbols 2p and 2p+1 of its group s), so in
// every round the lanes that need a word read CONSECUTIVE words: the wave
// ballots the request, each lane's word index is the popcount of the
// requesting lanes below it, and the wave's read cursor advances by the
// ballot's popcount.  The words pass through a ring in LDS refilled half a
// ring ahead with coalesced loads.
//
// A ZG stream (zero-aware coding of deltas) adds a bitmap of the groups that
// hold a value other than the fill value z: unmarked groups are z and take no
// part.  The 64 bits of one step of a lane group are contiguous in the
// bitmap; for a batch of 32 steps from J, lane l holds half l/32 of the bits
// of step J + l%32 (one register per stream), and every step reads its two
// halves with v_readlane.
//
// Any failed check records ZIPNN_E_CORRUPT / ZIPNN_E_FORMAT in the sticky
// status word; the decoder never reads outside [src, src+total_bytes) and
// never writes outside dst[0, n*B).
#include "zipnn_internal.h"

namespace zipnn {
namespace {

struct ItemState {
    uint64_t pay[4];       // absolute offset of each stream's payload in src
    uint32_t bytes[4];
    uint32_t mode[4];
    uint32_t rle[4];
    int err;
};

struct LutTmp {
    uint32_t nz, kraft, bad;
    uint32_t cnt[4][16];   // per-wave count of each code length
    uint32_t first[16];    // first canonical code of each length
    uint32_t offs[16];     // sorted position of the first code of each length
    uint16_t start[256];   // left-justified code of sorted position p
    uint16_t entry[256];   // symbol | length << 8 at sorted position p
    uint32_t red[8];
};

struct TensorState {
    Header h;
    int desc;
    int valid;
    ItemPlan p;
};

__device__ inline void set_status(int* st, int code) { atomicCAS(st, 0, code); }

__device__ inline uint32_t wave_incl_scan(uint32_t v)
{
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        uint32_t o = __shfl_up(v, d, 64);
        if (lane >= d) v += o;
    }
    return v;
}

// Expand a 128-byte nibble table into the LSB-first lookup table `lut`
// (entry = length | symbol << 8 for every L-bit window: bits 5..7 are zero, so
// a shift by the entry shifts by the length).  Returns false (in every
// thread) when the lengths are not a complete prefix code.
__device__ bool build_lut(const uint8_t* table, uint32_t L, uint16_t* lut, LutTmp& T)
{
    const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
    if (t < 16) {
        T.cnt[0][t] = T.cnt[1][t] = T.cnt[2][t] = T.cnt[3][t] = 0;
    }
    if (t == 0) T.nz = T.kraft = T.bad = 0;
    __syncthreads();
    const uint32_t b = table[t >> 1];
    const uint32_t l = (t & 1) ? (b >> 4) : (b & 15u);
    if (l > L) atomicOr(&T.bad, 1u);
    if (l && l <= L) {
        atomicAdd(&T.nz, 1u);
        atomicAdd(&T.kraft, 1u << (L - l));
    }
    const uint64_t lt_mask = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    uint32_t rank = 0;
    for (uint32_t len = 1; len <= L; len++) {
        uint64_t msk = __ballot(l == len);
        if (l == len) rank = __popcll(msk & lt_mask);
        if (lane == 0) T.cnt[wv][len] = __popcll(msk);
    }
    __syncthreads();
    if (t == 0) {
        uint32_t code = 0, prev = 0, off = 0;
        for (uint32_t len = 1; len <= L; len++) {
            code = (code + prev) << 1;
            uint32_t c = T.cnt[0][len] + T.cnt[1][len] + T.cnt[2][len] + T.cnt[3][len];
            T.first[len] = code;
            T.offs[len] = off;
            off += c;
            prev = c;
        }
    }
    __syncthreads();
    const bool ok = T.bad == 0 && T.nz >= 2 && T.kraft == (1u << L);
    if (!ok) return false;
    if (l) {
        uint32_t pre = 0;
        for (int i = 0; i < wv; i++) pre += T.cnt[i][l];
        uint32_t pos = T.offs[l] + pre + rank;
        uint32_t code = T.first[l] + pre + rank;
        T.start[pos] = uint16_t(code << (L - l));
        T.entry[pos] = uint16_t(l | (t << 8));
    }
    __syncthreads();
    // every L-bit value v (most significant code bit first) lies in the range
    // of exactly one sorted code: the last one whose left-justified code <= v
    const uint32_t nz = T.nz;
    const uint32_t per = (1u << L) / kBlock;
    const uint32_t v0 = t * per;
    uint32_t lo = 0, hi = nz - 1;
    while (lo < hi) {
        uint32_t mid = (lo + hi + 1) >> 1;
        if (T.start[mid] <= v0) lo = mid;
        else hi = mid - 1;
    }
    uint32_t p = lo;
    for (uint32_t v = v0; v < v0 + per; v++) {
        while (p + 1 < nz && T.start[p + 1] <= v) p++;
        lut[__brev(v) >> (32 - L)] = T.entry[p];
    }
    __syncthreads();
    return true;
}

typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

// Buffer resource over [p, p + bytes): loads past the end return zero and
// stores past it are dropped.  Offsets of accesses that must not happen are
// set to kOff, far past any valid range.
constexpr uint32_t kOff = 0x80000000u;

// Values the same in every lane of the wave, made scalar.
__device__ inline uint32_t uni(uint32_t v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ inline uint64_t uni64(uint64_t v)
{
    return uint64_t(uni(uint32_t(v))) | (uint64_t(uni(uint32_t(v >> 32))) << 32);
}
template <class T>
__device__ inline T* uniptr(T* p)
{
    return reinterpret_cast<T*>(uni64(reinterpret_cast<uint64_t>(p)));
}
__device__ inline __amdgpu_buffer_rsrc_t rsrc(const void* p, uint32_t bytes)
{
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), (short)0, (int)bytes, 0x00020000);
}

template <int NBYTES>
__device__ inline void buf_load(__amdgpu_buffer_rsrc_t r, uint32_t off, uint32_t* o)
{
    if constexpr (NBYTES == 2) o[0] = __builtin_amdgcn_raw_buffer_load_b16(r, off, 0, 2);
    else if constexpr (NBYTES == 4) o[0] = __builtin_amdgcn_raw_buffer_load_b32(r, off, 0, 2);
    else if constexpr (NBYTES == 8) {
        u32x2 v = __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, 2);
        o[0] = v.x;
        o[1] = v.y;
    } else if constexpr (NBYTES == 16) {
        u32x4 v = __builtin_amdgcn_raw_buffer_load_b128(r, off, 0, 2);
        o[0] = v.x;
        o[1] = v.y;
        o[2] = v.z;
        o[3] = v.w;
    } else {
        u32x4 v = __builtin_amdgcn_raw_buffer_load_b128(r, off, 0, 2);
        u32x4 u = __builtin_amdgcn_raw_buffer_load_b128(r, off + 16, 0, 2);
        o[0] = v.x;
        o[1] = v.y;
        o[2] = v.z;
        o[3] = v.w;
        o[4] = u.x;
        o[5] = u.y;
        o[6] = u.z;
        o[7] = u.w;
    }
}

template <int NBYTES>
__device__ inline void buf_store(__amdgpu_buffer_rsrc_t r, uint32_t off, const uint32_t* w)
{
    if constexpr (NBYTES == 2) __builtin_amdgcn_raw_buffer_store_b16(uint16_t(w[0]), r, off, 0, 2);
    else if constexpr (NBYTES == 4) __builtin_amdgcn_raw_buffer_store_b32(w[0], r, off, 0, 2);
    else if constexpr (NBYTES == 8) __builtin_amdgcn_raw_buffer_store_b64(u32x2{w[0], w[1]}, r, off, 0, 2);
    else if constexpr (NBYTES == 16) __builtin_amdgcn_raw_buffer_store_b128(u32x4{w[0], w[1], w[2], w[3]}, r, off, 0, 2);
    else {
        __builtin_amdgcn_raw_buffer_store_b128(u32x4{w[0], w[1], w[2], w[3]}, r, off, 0, 2);
        __builtin_amdgcn_raw_buffer_store_b128(u32x4{w[4], w[5], w[6], w[7]}, r, off + 16, 0, 2);
    }
}

constexpr int kDepth = 4;   // groups of raw bytes prefetched ahead per lane

// Words of a lane group's Huffman stream pass through a ring in LDS (per
// wave and stream) of RW words: two halves of RW/2.  When the read cursor has
// used up the older half, the block fetched one half earlier (held per lane
// in registers) is written there and the next block is fetched, so a fetch
// has a whole half of the ring's consumption to arrive.
template <int B>
struct Ring {
    static constexpr int RW = B == 4 ? 256 : 512;   // words per ring
    static constexpr int PN = RW / 128;             // words per lane of a pending half block
    static constexpr int CHECK = RW / 128;          // rounds between refill checks, at most
};

template <int B, int G>
struct SlotSize {
    static constexpr int PW = G >= 4 ? G / 4 : 1;                 // packed words per group
    static constexpr int HUF = Ring<B>::PN + 3;                   // pending block, count, 64-bit buffer
    static constexpr int N = kDepth * PW > HUF ? kDepth * PW : HUF;
};

// Uniform (scalar) state of a lane group's Huffman word stream.
struct WordCursor {
    __amdgpu_buffer_rsrc_t rs;   // this lane group's words
    uint32_t* ring;              // this wave's ring for the stream (LDS)
    uint8_t* rings;              // the workgroup's rings, aligned to RW*4 bytes
    uint32_t roff;               // byte offset of `ring` in `rings` (a multiple of RW*4)
    uint32_t ptr;                // words taken so far
    uint32_t rb;                 // stream index of the ring's oldest word (multiple of RW/2)
};

// A stream's register slot holds, for a Huffman stream: the pending block
// r[0..PN), the count r[PN] and the 64-bit bit buffer r[PN+1] | r[PN+2] << 32
// whose bit 0 is a placeholder: with c = r[PN] & 0xFF, the buffered code bits
// are bits 1 .. c-1, next code first, so that r[PN+1] & (table mask << 1) is
// the byte offset of the next code's table entry.  Decoding subtracts whole
// table entries from r[PN]: c loses the length, and the symbol bits only
// reach bits 8 and up (c stays within 1..55 and never borrows); for a raw
// stream: the ring of prefetched groups (r[u*PW + x]).  The mode of a stream is fixed for a chunk, so one set of
// registers serves both.

template <int B>
__device__ inline void pend_load(uint32_t* r, const WordCursor& c, uint32_t first, uint32_t lane)
{
    constexpr int PN = Ring<B>::PN;
    buf_load<4 * PN>(c.rs, (first + PN * lane) * 4, r);
}

template <int B>
__device__ inline void huf_init(uint32_t* r, WordCursor& c, const uint32_t* words, uint32_t nwords, uint32_t lane,
                                uint32_t* rings, uint32_t ring_index)
{
    constexpr int RW = Ring<B>::RW, PN = Ring<B>::PN;
    uint32_t* ring = rings + ring_index * RW;
    c.rs = rsrc(words, nwords * 4);
    c.ring = ring;
    c.rings = reinterpret_cast<uint8_t*>(rings);
    c.roff = ring_index * RW * 4;
    c.ptr = 0;
    c.rb = 0;
    // fill the ring with words [0, RW), then fetch [RW, RW + RW/2)
    uint32_t v[2 * PN];
    buf_load<8 * PN>(c.rs, 2 * PN * lane * 4, v);
#pragma unroll
    for (int x = 0; x < 2 * PN; x++) ring[2 * PN * lane + x] = v[x];
    pend_load<B>(r, c, RW, lane);
    r[PN] = 1;   // no code bits yet, only the placeholder bit
    r[PN + 1] = 0;
    r[PN + 2] = 0;
}

// One round's word requests: lanes taking part with fewer than 2L buffered
// bits (r[PN] <= 2L) take the next words of the stream, in lane order (a
// ballot and a prefix popcount give each lane its word).
template <int B>
__device__ inline void huf_take(uint32_t* r, WordCursor& c, bool part, uint32_t twoL)
{
    constexpr int RW = Ring<B>::RW, PN = Ring<B>::PN;
    const bool need = part && (r[PN] & 0xFFu) <= twoL;
    const uint64_t m = __ballot(need);
    // this lane's word: the cursor plus the needing lanes below, modulo the
    // ring; the ring's byte offset is a multiple of its size, so OR places it
    const uint32_t below = __builtin_amdgcn_mbcnt_hi(uint32_t(m >> 32), __builtin_amdgcn_mbcnt_lo(uint32_t(m), 0u));
    const uint32_t off = ((c.ptr * 4u + below * 4u) & (RW * 4u - 4u)) | c.roff;
    const uint32_t word = *(const uint32_t*)(c.rings + off);   // every lane reads; only the needing ones keep it
    const uint64_t x = uint64_t(need ? word : 0u) << (r[PN] & 63u);
    r[PN + 1] |= uint32_t(x);
    r[PN + 2] |= uint32_t(x >> 32);
    r[PN] += need ? 32u : 0u;
    c.ptr += uint32_t(__popcll(m));
}

// Called at least every Ring<B>::CHECK rounds: a round takes at most 64
// words, so between checks the reads stay inside the ring's RW words.
template <int B>
__device__ inline void huf_refill(uint32_t* r, WordCursor& c, uint32_t lane)
{
    constexpr int RW = Ring<B>::RW, PN = Ring<B>::PN;
    if (c.ptr - c.rb >= RW / 2) {
        // the older half is used up: it receives the pending block
        uint32_t* half = c.ring + (c.rb & (RW - 1));
#pragma unroll
        for (int x = 0; x < PN; x++) half[PN * lane + x] = r[x];
        c.rb += RW / 2;
        pend_load<B>(r, c, c.rb + RW, lane);
    }
}

// Decode one symbol: returns its table entry (length | symbol << 8) and
// drops its code bits.  mask2 = (2^L - 1) << 1 picks the byte offset of the
// entry of the L bits after the placeholder; the funnel shifts use the low
// five bits of the entry, which are the length.
template <int B>
__device__ inline uint32_t huf_get(uint32_t* r, const uint16_t* lut, uint32_t mask2)
{
    constexpr int PN = Ring<B>::PN;
    const uint32_t e = *(const uint16_t*)((const uint8_t*)lut + (r[PN + 1] & mask2));
    r[PN + 1] = __builtin_amdgcn_alignbit(r[PN + 2], r[PN + 1], e);
    r[PN + 2] = __builtin_amdgcn_alignbit(0u, r[PN + 2], e);
    r[PN] -= e;
    return e;
}

// huf_get for a lane that may not take part (a ZG group made of z alone):
// the table is read, but the bits are consumed only when `on`.
template <int B>
__device__ inline uint32_t huf_get_if(uint32_t* r, const uint16_t* lut, uint32_t mask2, bool on)
{
    constexpr int PN = Ring<B>::PN;
    const uint32_t e = *(const uint16_t*)((const uint8_t*)lut + (r[PN + 1] & mask2));
    const uint32_t s = on ? e : 0u;
    r[PN + 1] = __builtin_amdgcn_alignbit(r[PN + 2], r[PN + 1], s);
    r[PN + 2] = __builtin_amdgcn_alignbit(0u, r[PN + 2], s);
    r[PN] -= s;
    return e;
}

// A pair of symbols in two halves.  huf_pair0 reads the first symbol's entry
// and returns it with `lo1`, the buffer's low word past its code; huf_pair1
// reads the second entry from lo1 and drops both codes at once (the sum of
// two entries carries the sum of the lengths, at most 2L < 32, in its low
// five bits).  With `on` false the lane consumes nothing.
template <int B>
__device__ inline uint32_t huf_pair0(const uint32_t* r, const uint16_t* lut, uint32_t mask2, uint32_t& lo1)
{
    constexpr int PN = Ring<B>::PN;
    const uint32_t e = *(const uint16_t*)((const uint8_t*)lut + (r[PN + 1] & mask2));
    lo1 = __builtin_amdgcn_alignbit(r[PN + 2], r[PN + 1], e);
    return e;
}
template <int B>
__device__ inline uint32_t huf_pair1(uint32_t* r, const uint16_t* lut, uint32_t mask2, uint32_t e0, uint32_t lo1,
                                     bool on = true)
{
    constexpr int PN = Ring<B>::PN;
    const uint32_t e1 = *(const uint16_t*)((const uint8_t*)lut + (lo1 & mask2));
    const uint32_t s = on ? e0 + e1 : 0u;
    r[PN + 1] = __builtin_amdgcn_alignbit(r[PN + 2], r[PN + 1], s);
    r[PN + 2] = __builtin_amdgcn_alignbit(0u, r[PN + 2], s);
    r[PN] -= s;
    return e1;
}

// The symbols of two table entries as bytes `pos` and pos+1 of a word whose
// other bytes are zero (v_perm_b32: selector 1 is byte 1 of the second
// operand, 5 byte 1 of the first, 0x0c a zero byte).
__device__ inline uint32_t sym_pair(uint32_t e0, uint32_t e1, uint32_t pos)
{
    return __builtin_amdgcn_perm(e1, e0, pos == 0 ? 0x0c0c0501u : 0x05010c0cu);
}

template <int G>
__device__ inline void raw_load(const uint8_t* p, uint32_t* o)
{
    if constexpr (G == 2) o[0] = *(const uint16_t*)p;
    else if constexpr (G == 4) o[0] = __builtin_nontemporal_load((const uint32_t*)p);
    else {
        u32x2 v = __builtin_nontemporal_load((const u32x2*)p);
        o[0] = v.x;
        o[1] = v.y;
    }
}

template <int NB>
__device__ inline void store_words(uint8_t* d, const uint32_t* w)
{
    if constexpr (NB == 2) *(uint16_t*)d = uint16_t(w[0]);
    else if constexpr (NB == 4) __builtin_nontemporal_store(w[0], (uint32_t*)d);
    else if constexpr (NB == 8) __builtin_nontemporal_store(u32x2{w[0], w[1]}, (u32x2*)d);
    else if constexpr (NB == 16) __builtin_nontemporal_store(u32x4{w[0], w[1], w[2], w[3]}, (u32x4*)d);
    else {
        __builtin_nontemporal_store(u32x4{w[0], w[1], w[2], w[3]}, (u32x4*)d);
        __builtin_nontemporal_store(u32x4{w[4], w[5], w[6], w[7]}, (u32x4*)(d + 16));
    }
}

template <int NB>
__device__ inline void load_words(const uint8_t* b, uint32_t* w)
{
    if constexpr (NB == 2) w[0] = *(const uint16_t*)b;
    else if constexpr (NB == 4) w[0] = __builtin_nontemporal_load((const uint32_t*)b);
    else {
#pragma unroll
        for (int i = 0; i < NB / 8; i++) {
            u32x2 v = __builtin_nontemporal_load((const u32x2*)(b + 8 * i));
            w[2 * i] = v.x;
            w[2 * i + 1] = v.y;
        }
    }
}

// Interleave the B byte groups of G elements back into words (the inverse of
// byte grouping): pk[k][x] holds symbols 4x..4x+3 of stream k; element i's
// little-endian word is (s_{B-1}[i], ..., s_1[i], s_0[i]).  v_perm_b32 picks
// bytes of {S0:S1} (selector 0-3: S1, 4-7: S0).
template <int B, int G>
__device__ inline void merge_words(const uint32_t (*pk)[G >= 4 ? G / 4 : 1], uint32_t* ow)
{
    constexpr int PW = G >= 4 ? G / 4 : 1;
    if constexpr (B == 1) {
#pragma unroll
        for (int x = 0; x < PW; x++) ow[x] = pk[0][x];
    } else if constexpr (B == 2) {
#pragma unroll
        for (int x = 0; x < PW; x++) {
            ow[2 * x] = __builtin_amdgcn_perm(pk[0][x], pk[1][x], 0x05010400u);
            if constexpr (G >= 4) ow[2 * x + 1] = __builtin_amdgcn_perm(pk[0][x], pk[1][x], 0x07030602u);
        }
    } else {
#pragma unroll
        for (int x = 0; x < PW; x++) {
            const uint32_t lo01 = __builtin_amdgcn_perm(pk[0][x], pk[1][x], 0x05010400u);
            const uint32_t lo23 = __builtin_amdgcn_perm(pk[2][x], pk[3][x], 0x05010400u);
            ow[4 * x] = __builtin_amdgcn_perm(lo01, lo23, 0x05040100u);
            ow[4 * x + 1] = __builtin_amdgcn_perm(lo01, lo23, 0x07060302u);
            if constexpr (G >= 4) {
                const uint32_t hi01 = __builtin_amdgcn_perm(pk[0][x], pk[1][x], 0x07030602u);
                const uint32_t hi23 = __builtin_amdgcn_perm(pk[2][x], pk[3][x], 0x07030602u);
                ow[4 * x + 2] = __builtin_amdgcn_perm(hi01, hi23, 0x05040100u);
                ow[4 * x + 3] = __builtin_amdgcn_perm(hi01, hi23, 0x07060302u);
            }
        }
    }
}

// Decode lane group j of one chunk: every stream's symbols of the lane's
// sub-stream, merged into words and stored.  Raw bytes (and the XOR base) of
// a lane's groups are fetched kDepth groups ahead through a register ring.
// While every lane of the group still has a full group of g symbols the loop
// runs without per-lane conditions; the last groups take the general path.
template <int B, int G, bool DELTA, bool ZGK>
__device__ __attribute__((always_inline)) void decode_lane_group(const uint8_t* __restrict__ src, const ItemState& st, uint32_t* wring,
                                  const uint16_t (*lut)[kLutSize], const uint32_t (*wprefix)[65], uint32_t L,
                                  uint32_t j, uint32_t W, uint32_t m, uint8_t* __restrict__ out,
                                  const uint8_t* __restrict__ base, int* status, bool xf)
{
    constexpr int NB = B * G;
    constexpr int NW = NB >= 4 ? NB / 4 : 1;
    constexpr int PW = SlotSize<B, G>::PW;
    constexpr int NS = SlotSize<B, G>::N;
    constexpr int BD = DELTA ? kDepth : 1;
    src = uniptr(src);
    out = uniptr(out);
    base = uniptr(base);
    j = uni(j);
    W = uni(W);
    m = uni(m);
    L = uni(L);
    const uint32_t lane = threadIdx.x & 63;
    const uint32_t w = 64 * j + lane;
    const uint32_t mask2 = ((1u << L) - 1) << 1, twoL = 2 * L;
    const uint32_t Gtot = (m + G - 1) / G, Gfull = m / G, rem = m - Gfull * G;
    const uint32_t ng = (w < W && w < Gtot) ? (Gtot - 1 - w) / W + 1 : 0;     // groups of this lane
    const uint32_t nfull = (w < W && w < Gfull) ? (Gfull - 1 - w) / W + 1 : 0; // full ones
    const uint32_t ng_max = __builtin_amdgcn_readfirstlane(ng);            // lane 0 has the most
    // full groups of the last lane of the group: every lane has at least these
    const uint32_t w_last = min(W, 64 * j + 64) - 1;
    const uint32_t nfull_all = w_last < Gfull ? (Gfull - 1 - w_last) / W + 1 : 0;
    uint32_t n_fast = (64 * j + 64 <= W) ? nfull_all / kDepth * kDepth : 0;
    int mode[B];
    uint32_t rlev[B];
    const uint8_t* pay[B];
    __amdgpu_buffer_rsrc_t rr[B];
    WordCursor cur[B];
    uint32_t nw[B];
    uint32_t slot[B][NS];
    uint32_t bring[BD][NW];
    uint32_t zwin[B];   // ZG: bits of the current batch of 32 steps
    uint32_t zJ = 0;    // first step of the batch
    const __amdgpu_buffer_rsrc_t ro = rsrc(out, m * B);
    const __amdgpu_buffer_rsrc_t rb = rsrc(DELTA ? base : out, m * B);
    // byte offset of this lane's group jj in a raw payload: (w + jj*W)*G
    auto raw_off = [&](uint32_t jj) { return jj < nfull ? (w + jj * W) * G : kOff; };
    // the same for the XOR base, in bytes
    auto base_off = [&](uint32_t jj) { return jj < nfull ? (w + jj * W) * (G * B) : kOff; };
    // ZG: lane l loads bits 32(l/32) .. +31 of step J + l%32 of this lane
    // group, i.e. bits 64j + (J + l%32)W + 32(l/32) onwards of the bitmap
    auto zload = [&](int k, uint32_t J) __attribute__((always_inline)) {
        const __amdgpu_buffer_rsrc_t zr = rsrc(pay[k] + huf_head(W), zg_bitmap(m, G));
        const uint32_t s = J + (lane & 31);
        const uint32_t b0 = 64 * j + s * W + 32 * (lane >> 5);
        const uint32_t o = s < ng_max ? (b0 >> 5) * 4 : kOff;
        uint32_t d0, d1;
        buf_load<4>(zr, o, &d0);
        buf_load<4>(zr, o == kOff ? kOff : o + 4, &d1);
        zwin[k] = __builtin_amdgcn_alignbit(d1, d0, b0 & 31);
    };
#pragma unroll
    for (int k = 0; k < B; k++) {
        mode[k] = __builtin_amdgcn_readfirstlane(st.mode[k]);
        rlev[k] = st.rle[k] * 0x01010101u;
        pay[k] = src + uni64(st.pay[k]);
        rr[k] = rsrc(pay[k], mode[k] == kModeRaw ? m : 0u);
#pragma unroll
        for (int x = 0; x < NS; x++) slot[k][x] = 0;
        zwin[k] = 0;
        const bool zg = (ZGK && mode[k] == kModeZg);
        const uint32_t bm = zg ? zg_bitmap(m, G) : 0u;
        if (zg) zload(k, 0);
        if (mode[k] == kModeHuf || zg) {
            const uint32_t* words = (const uint32_t*)(pay[k] + huf_head(W) + bm);
            const uint32_t s0 = __builtin_amdgcn_readfirstlane(wprefix[k][j]);
            const uint32_t s1 = __builtin_amdgcn_readfirstlane(wprefix[k][j + 1]);
            nw[k] = s1 - s0;
            huf_init<B>(slot[k], cur[k], words + s0, s1 - s0, lane, wring, k * 4 + (threadIdx.x >> 6));
        } else if (mode[k] == kModeRaw) {
#pragma unroll
            for (int u = 0; u < kDepth; u++) buf_load<G>(rr[k], raw_off(u), &slot[k][u * PW]);
        }
    }
    if constexpr (DELTA) {
#pragma unroll
        for (int u = 0; u < kDepth; u++) {
            buf_load<NB>(rb, base_off(u), bring[u]);
        }
    }
    // ZG: at step jj (the steps are visited in order, kDepth at a time),
    // whether this lane's group is marked; every 32 steps the next batch of
    // bits is loaded
    auto zstep = [&](uint32_t jj, uint32_t zm) __attribute__((always_inline)) {
        if (jj == zJ + 32) {
            zJ += 32;
#pragma unroll
            for (int k = 0; k < B; k++)
                if ((zm >> k) & 1) zload(k, zJ);
        }
    };
    // the 64 group bits of step jj (uniform; bits of lanes past W belong to
    // other steps' groups)
    auto zmask = [&](int k, uint32_t jj) __attribute__((always_inline)) {
        const uint32_t sidx = uni(jj - zJ);
        const uint32_t lo = __builtin_amdgcn_readlane(zwin[k], sidx);
        const uint32_t hi = __builtin_amdgcn_readlane(zwin[k], sidx + 32);
        return uint64_t(lo) | (uint64_t(hi) << 32);
    };
    uint32_t zm_all = 0;
#pragma unroll
    for (int k = 0; k < B; k++) zm_all |= uint32_t((ZGK && mode[k] == kModeZg)) << k;
    // fast path: all 64 lanes have full groups j0 .. j0+kDepth-1.  HM is the
    // set of Huffman and ZG streams and ZM that of the ZG ones, or -1 for sets
    // without their own copy of the loop, tested per stream at run time; the
    // other streams are raw or single-valued (a uniform test per step).
    auto fast = [&](auto hm_const, auto zm_const) __attribute__((always_inline)) {
        constexpr int HM = decltype(hm_const)::value;
        constexpr int ZM = decltype(zm_const)::value;
        // the interleaved form below (HM >= 0, B <= 2): ZS, the ZG streams
        // decoded there; CM, all the streams it decodes
        constexpr int ZS = (ZM >= 0 && !DELTA) ? ZM : 0;
        constexpr int CM = HM & ~((ZM >= 0 ? ZM : 0) & ~ZS);
        // both byte groups of a BF16/FP16 word coded: the words are built
        // from the table entries directly
        constexpr bool DIRECT = HM >= 0 && B == 2 && CM == 3 && ZS == 0;
        for (uint32_t j0 = 0; j0 < n_fast; j0 += kDepth) {
#pragma unroll
            for (int u = 0; u < kDepth; u++) {
                const uint32_t jj = j0 + u;
                const uint32_t off = (w + jj * W) * G;
                const uint32_t offn = raw_off(jj + kDepth);
                if (ZM != 0 && u == 0) zstep(jj, ZM >= 0 ? uint32_t(ZM) : zm_all);
                uint32_t pk[B][PW];
                uint32_t ow[NW];
                bool zon[B];   // ZG streams decoded side by side: this lane's group is marked
#pragma unroll
                for (int k = 0; k < B; k++) {
                    const bool is_huf = HM >= 0 ? ((HM >> k) & 1) != 0 : (mode[k] == kModeHuf || (ZGK && mode[k] == kModeZg));
                    const bool is_zg = ZM >= 0 ? ((ZM >> k) & 1) != 0 : (ZGK && mode[k] == kModeZg);
                    zon[k] = false;
                    if (HM >= 0 && B <= 2 && !DELTA && is_zg) {
                        zon[k] = ((zmask(k, jj) >> lane) & 1) != 0;
#pragma unroll
                        for (int x = 0; x < PW; x++) pk[k][x] = 0;
                    } else if (!is_huf) {
                        // raw, or a single value filled from a register (its
                        // buffer has no bytes, so its loads read nothing)
                        const bool rle = mode[k] == kModeRle;
#pragma unroll
                        for (int x = 0; x < PW; x++) pk[k][x] = rle ? rlev[k] : slot[k][u * PW + x];
                        buf_load<G>(rr[k], offn, &slot[k][u * PW]);
                    } else if (is_zg) {
                        const uint64_t zm = zmask(k, jj);
#pragma unroll
                        for (int x = 0; x < PW; x++) pk[k][x] = rlev[k];
                        if (zm != 0) {   // else no lane of the wave takes part in this step
                            const bool on = ((zm >> lane) & 1) != 0;
#pragma unroll
                            for (int x = 0; x < PW; x++) pk[k][x] = 0;
#pragma unroll
                            for (int pr = 0; pr < G / 2; pr++) {
                                huf_take<B>(slot[k], cur[k], on, twoL);
                                uint32_t lo1;
                                const uint32_t e0 = huf_pair0<B>(slot[k], lut[k], mask2, lo1);
                                const uint32_t e1 = huf_pair1<B>(slot[k], lut[k], mask2, e0, lo1, on);
                                pk[k][(2 * pr) >> 2] |= sym_pair(e0, e1, (2 * pr) & 3);
                                if ((pr + 1) % Ring<B>::CHECK == 0 || pr == G / 2 - 1)
                                    huf_refill<B>(slot[k], cur[k], lane);
                            }
#pragma unroll
                            for (int x = 0; x < PW; x++) pk[k][x] = on ? pk[k][x] : rlev[k];
                        }
                    } else {
#pragma unroll
                        for (int x = 0; x < PW; x++) pk[k][x] = 0;
                        if constexpr (HM < 0 || B > 2) {
                            // stream by stream (a set known at run time only,
                            // or 4-byte words, where the interleaved form
                            // below measured slower)
#pragma unroll
                            for (int pr = 0; pr < G / 2; pr++) {
                                huf_take<B>(slot[k], cur[k], true, twoL);
                                uint32_t lo1;
                                const uint32_t e0 = huf_pair0<B>(slot[k], lut[k], mask2, lo1);
                                const uint32_t e1 = huf_pair1<B>(slot[k], lut[k], mask2, e0, lo1);
                                pk[k][(2 * pr) >> 2] |= sym_pair(e0, e1, (2 * pr) & 3);
                                if ((pr + 1) % Ring<B>::CHECK == 0 || pr == G / 2 - 1)
                                    huf_refill<B>(slot[k], cur[k], lane);
                            }
                        }
                    }
                }
                if constexpr (HM >= 0 && B <= 2) {
                    // the coded streams (a set fixed at compile time) pair by
                    // pair, every stream's step of a pair next to the others':
                    // the chains of table reads of the streams overlap (BF16
                    // chunks with both groups coded: -7%).  In a ZG stream the
                    // lanes whose group is z alone take no part.
                    uint32_t ent[B][G];
#pragma unroll
                    for (int pr = 0; pr < G / 2; pr++) {
                        uint32_t e0[B], lo1[B];
#pragma unroll
                        for (int k = 0; k < B; k++)
                            if ((CM >> k) & 1) huf_take<B>(slot[k], cur[k], ((ZS >> k) & 1) ? zon[k] : true, twoL);
#pragma unroll
                        for (int k = 0; k < B; k++) {
                            if ((CM >> k) & 1) e0[k] = huf_pair0<B>(slot[k], lut[k], mask2, lo1[k]);
                        }
#pragma unroll
                        for (int k = 0; k < B; k++) {
                            if ((CM >> k) & 1) {
                                const uint32_t e1 = huf_pair1<B>(slot[k], lut[k], mask2, e0[k], lo1[k],
                                                                 ((ZS >> k) & 1) ? zon[k] : true);
                                ent[k][2 * pr] = e0[k];
                                ent[k][2 * pr + 1] = e1;
                                if (!DIRECT) pk[k][(2 * pr) >> 2] |= sym_pair(e0[k], e1, (2 * pr) & 3);
                            }
                        }
#pragma unroll
                        for (int k = 0; k < B; k++)
                            if (((CM >> k) & 1) && ((pr + 1) % Ring<B>::CHECK == 0 || pr == G / 2 - 1))
                                huf_refill<B>(slot[k], cur[k], lane);
                    }
#pragma unroll
                    for (int k = 0; k < B; k++)
                        if ((ZS >> k) & 1)
#pragma unroll
                            for (int x = 0; x < PW; x++) pk[k][x] = zon[k] ? pk[k][x] : rlev[k];
                    if constexpr (DIRECT) {
                        // word x holds elements 2x (bytes 0, 1) and 2x+1: the
                        // low byte from group 1, the high byte from group 0
#pragma unroll
                        for (int x = 0; x < G / 2; x++)
                            ow[x] = __builtin_amdgcn_perm(ent[0][2 * x], ent[1][2 * x], 0x0c0c0501u) |
                                    __builtin_amdgcn_perm(ent[0][2 * x + 1], ent[1][2 * x + 1], 0x05010c0cu);
                    }
                }
                if constexpr (!DIRECT) merge_words<B, G>(pk, ow);
                if (xf)
#pragma unroll
                    for (int x = 0; x < NW; x++) ow[x] = exp_inv<B>(ow[x]);
                if constexpr (DELTA) {
#pragma unroll
                    for (int x = 0; x < NW; x++) ow[x] ^= bring[u][x];
                    buf_load<NB>(rb, base_off(jj + kDepth), bring[u]);
                }
                buf_store<NB>(ro, off * B, ow);
            }
        }
    };
    {
        uint32_t hm = 0;
#pragma unroll
        for (int k = 0; k < B; k++) hm |= uint32_t(mode[k] == kModeHuf || (ZGK && mode[k] == kModeZg)) << k;
        const uint32_t zm = zm_all;
        using std::integral_constant;
        using I = int;
        // a copy of the loop for every set of a BF16/FP8 chunk and for the
        // common FP32 sets (ZM != 0 only in the kernels with the ZG decoder)
        auto spec = [&](auto h, auto z) {
            constexpr int H = decltype(h)::value, Z = decltype(z)::value;
            if constexpr (Z != 0 && !ZGK) return false;
            else {
                if (hm != uint32_t(H) || zm != uint32_t(Z)) return false;
                fast(h, z);
                return true;
            }
        };
        bool done = false;
        if constexpr (B == 1) {
            done = spec(integral_constant<I, 0>{}, integral_constant<I, 0>{}) ||
                   spec(integral_constant<I, 1>{}, integral_constant<I, 0>{}) ||
                   spec(integral_constant<I, 1>{}, integral_constant<I, 1>{});
        } else if constexpr (B == 2) {
            done = spec(integral_constant<I, 0>{}, integral_constant<I, 0>{}) ||
                   spec(integral_constant<I, 1>{}, integral_constant<I, 0>{}) ||
                   spec(integral_constant<I, 2>{}, integral_constant<I, 0>{}) ||
                   spec(integral_constant<I, 3>{}, integral_constant<I, 0>{}) ||
                   spec(integral_constant<I, 1>{}, integral_constant<I, 1>{}) ||
                   spec(integral_constant<I, 2>{}, integral_constant<I, 2>{}) ||
                   spec(integral_constant<I, 3>{}, integral_constant<I, 1>{}) ||
                   spec(integral_constant<I, 3>{}, integral_constant<I, 2>{}) ||
                   spec(integral_constant<I, 3>{}, integral_constant<I, 3>{});
        } else {
            done = spec(integral_constant<I, 0>{}, integral_constant<I, 0>{}) ||
                   spec(integral_constant<I, 1>{}, integral_constant<I, 0>{}) ||
                   spec(integral_constant<I, 3>{}, integral_constant<I, 0>{}) ||
                   spec(integral_constant<I, 1>{}, integral_constant<I, 1>{}) ||
                   spec(integral_constant<I, 3>{}, integral_constant<I, 3>{}) ||
                   spec(integral_constant<I, 15>{}, integral_constant<I, 15>{});
        }
        if (!done) fast(integral_constant<I, -1>{}, integral_constant<I, -1>{});
    }
    // general path: the remaining groups, with per-lane conditions
    for (uint32_t j0 = n_fast; j0 < ng_max; j0 += kDepth) {
#pragma unroll
        for (int u = 0; u < kDepth; u++) {
            const uint32_t jj = j0 + u;
            const uint32_t q = w + jj * W;
            const bool has = jj < ng;
            const bool full = jj < nfull;
            const uint32_t gcnt = full ? G : (has ? rem : 0);
            const uint32_t offn = raw_off(jj + kDepth);
            if (zm_all && u == 0) zstep(jj, zm_all);
            uint32_t pk[B][PW];
#pragma unroll
            for (int k = 0; k < B; k++) {
#pragma unroll
                for (int x = 0; x < PW; x++) pk[k][x] = 0;
                // a ZG group made of z alone takes no part in the rounds.  The
                // flag is read with every lane active (a branch on `has` could
                // reload the window for some lanes only, and v_readlane would
                // then read a lane that was not loaded).
                const bool zg = ZGK && mode[k] == kModeZg;
                const bool flag = zg ? ((zmask(k, jj) >> lane) & 1) != 0 : true;
                const bool on = !zg || (has & flag);
                if (mode[k] == kModeRaw) {
#pragma unroll
                    for (int x = 0; x < PW; x++) pk[k][x] = slot[k][u * PW + x];
                    buf_load<G>(rr[k], offn, &slot[k][u * PW]);
                } else if (mode[k] == kModeRle) {
#pragma unroll
                    for (int x = 0; x < PW; x++) pk[k][x] = rlev[k];
                } else {
#pragma unroll
                    for (int pr = 0; pr < G / 2; pr++) {
                        const bool part = on && 2u * pr < gcnt;
                        huf_take<B>(slot[k], cur[k], part, twoL);
                        if (part) {
                            pk[k][(2 * pr) >> 2] |= (huf_get<B>(slot[k], lut[k], mask2) >> 8) << (8 * ((2 * pr) & 3));
                            if (2u * pr + 1 < gcnt)
                                pk[k][(2 * pr + 1) >> 2] |= (huf_get<B>(slot[k], lut[k], mask2) >> 8)
                                                            << (8 * ((2 * pr + 1) & 3));
                        }
                        if ((pr + 1) % Ring<B>::CHECK == 0 || pr == G / 2 - 1) huf_refill<B>(slot[k], cur[k], lane);
                    }
                    if (!on) {
#pragma unroll
                        for (int x = 0; x < PW; x++) pk[k][x] = rlev[k];
                    }
                }
            }
            uint32_t ow[NW];
            merge_words<B, G>(pk, ow);
            if (xf)
#pragma unroll
                for (int x = 0; x < NW; x++) ow[x] = exp_inv<B>(ow[x]);
            if constexpr (DELTA) {
#pragma unroll
                for (int x = 0; x < NW; x++) ow[x] ^= bring[u][x];
                buf_load<NB>(rb, base_off(jj + kDepth), bring[u]);
            }
            if (full) {
                buf_store<NB>(ro, q * G * B, ow);
            } else if (has) {
                // the partial last group of a tensor: one element at a time
                const uint32_t e = q * G;
                for (uint32_t i = 0; i < gcnt; i++) {
                    uint32_t word = 0;
#pragma unroll
                    for (int b = 0; b < B; b++) {
                        const int k = B - 1 - b;
                        uint32_t v;
                        if (mode[k] == kModeRaw) v = pay[k][e + i];
                        else {
                            v = pk[k][0];
#pragma unroll
                            for (int x = 1; x < PW; x++)
                                if (i >= 4u * x) v = pk[k][x];
                            v = (v >> (8 * (i & 3))) & 0xFFu;
                        }
                        word |= v << (8 * b);
                    }
                    if (xf) word = exp_inv<B>(word);
#pragma unroll
                    for (int b = 0; b < B; b++) {
                        const uint64_t o = uint64_t(e + i) * B + b;
                        const uint32_t v = (word >> (8 * b)) & 0xFFu;
                        out[o] = DELTA ? uint8_t(v ^ base[o]) : uint8_t(v);
                    }
                }
            }
        }
    }
#pragma unroll
    for (int k = 0; k < B; k++)
        if ((mode[k] == kModeHuf || (ZGK && mode[k] == kModeZg)) && cur[k].ptr != nw[k] && lane == 0)
            set_status(status, ZIPNN_E_CORRUPT);
}

// Parse one tensor's header on the device and size its work.
__device__ bool load_tensor(const DecDesc& d, int di, TensorState& ts, int* status, bool report)
{
    const uint4* hp = (const uint4*)d.src;
    uint32_t w[16];
    int rc = ZIPNN_OK;
    if (d.src_len < 64) rc = ZIPNN_E_FORMAT;
    if (rc == ZIPNN_OK) {
#pragma unroll
        for (int i = 0; i < 4; i++) {
            uint4 v = hp[i];
            w[4 * i] = v.x;
            w[4 * i + 1] = v.y;
            w[4 * i + 2] = v.z;
            w[4 * i + 3] = v.w;
        }
        rc = parse_header(w, d.src_len, ts.h);
    }
    if (rc == ZIPNN_OK) {
        const bool delta = ts.h.flags & kFlagDelta;
        if (delta != (d.base != nullptr)) rc = ZIPNN_E_FORMAT;
        else if (ts.h.n * ts.h.B > d.dst_cap) rc = ZIPNN_E_NOSPACE;
    }
    ts.desc = di;
    ts.valid = rc == ZIPNN_OK;
    ts.p.items = 0;
    if (rc != ZIPNN_OK) {
        if (report) set_status(status, rc);
        return false;
    }
    ts.p = plan_items(ts.h, d.c_begin, d.c_end);
    return true;
}

// One item: the B map entries are checked, each Huffman table becomes an LDS
// lookup table, the lane groups' word counts are checked and prefixed, then
// every wave decodes its lane group.
template <int B, int G, bool DELTA, bool ZGK>
__device__ __attribute__((always_inline)) void decode_item(const DecDesc& d, const TensorState& ts, uint32_t c, uint32_t slice, uint32_t* wring,
                            uint16_t (*lut)[kLutSize], uint32_t (*wprefix)[65], LutTmp& T, ItemState& st,
                            int* status)
{
    const Header& h = ts.h;
    const int t = threadIdx.x;
    const uint32_t m = uint32_t(min(uint64_t(h.E), h.n - uint64_t(c) * h.E));
    const uint32_t W = (m + h.S - 1) / h.S;
    const uint32_t NG = (W + 63) / 64;
    if (t == 0) st.err = 0;
    __syncthreads();
    if (t < B) {
        const uint64_t e = uint64_t(c) * B + t;
        const uint4 ent = *(const uint4*)(d.src + 64 + 16 * e);
        const uint64_t off = uint64_t(ent.x) | (uint64_t(ent.y) << 32);
        const uint32_t bytes = ent.z;
        const uint32_t mode = ent.w & 0xFF, rle = (ent.w >> 8) & 0xFF;
        int err = 0;
        if ((ent.w >> 16) != 0 || mode > 3) err = 1;
        if (mode == kModeRaw && (bytes != m || rle)) err = 1;
        if (mode == kModeRle && bytes != 0) err = 1;
        if (mode == kModeHuf && (bytes < huf_head(W) + 4 || ((bytes - huf_head(W)) & 3) || rle)) err = 1;
        if (mode == kModeZg && (!ZGK || !(h.flags & kFlagZg) || bytes < huf_head(W) + zg_bitmap(m, h.g) ||
                                ((bytes - huf_head(W)) & 3)))
            err = 1;
        if (off & (kPayAlign - 1)) err = 1;
        // the exact placement: this entry starts where its predecessor ends
        uint64_t expect = 0;
        if (e > 0) {
            const uint4 pe = *(const uint4*)(d.src + 64 + 16 * (e - 1));
            const uint64_t poff = uint64_t(pe.x) | (uint64_t(pe.y) << 32);
            expect = poff + align_pay(pe.z);
        }
        if (off != expect) err = 1;
        if (h.payload_base + off + bytes > h.total) err = 1;
        if (e + 1 == uint64_t(h.n_chunks) * B && h.payload_base + off + align_pay(bytes) != h.total) err = 1;
        st.pay[t] = h.payload_base + off;
        st.bytes[t] = bytes;
        st.mode[t] = mode;
        st.rle[t] = rle;
        if (err) {
            st.err = 1;
            set_status(status, ZIPNN_E_CORRUPT);
        }
    }
    __syncthreads();
    if (st.err) return;
    for (int k = 0; k < B; k++) {
        const bool zg = st.mode[k] == kModeZg;
        if (st.mode[k] != kModeHuf && !zg) continue;
        const uint8_t* p = d.src + st.pay[k];
        const uint32_t bm = zg ? zg_bitmap(m, h.g) : 0u;
        if (!build_lut(p, h.L, lut[k], T)) {
            if (t == 0) {
                st.err = 1;
                set_status(status, ZIPNN_E_CORRUPT);
            }
            __syncthreads();
            return;
        }
        // word counts of the lane groups -> start of each lane group's words;
        // in HUF every lane takes at least one word; together they use the
        // payload exactly.  A ZG bitmap has no bit past the last group.
        if (t < 64) {
            const uint32_t lanes_here = (uint32_t(t) < NG && !zg) ? min(64u, W - 64u * t) : 0u;
            const uint32_t nw = (uint32_t(t) < NG) ? ((const uint32_t*)(p + 128))[t] : 0u;
            const uint32_t inc = wave_incl_scan(nw);
            wprefix[k][t + 1] = inc;
            if (t == 0) wprefix[k][0] = 0;
            bool bad = nw < lanes_here;
            const uint32_t Gtot = (m + h.g - 1) / h.g;
            for (uint32_t i = Gtot / 8 + t; i < bm; i += 64) {
                uint32_t v = p[huf_head(W) + i];
                if (i == Gtot / 8) v &= ~((1u << (Gtot & 7)) - 1u);
                bad |= v != 0;
            }
            const uint32_t total = __shfl(inc, 63, 64);
            if (__ballot(bad) != 0ull || uint64_t(total) * 4 + huf_head(W) + bm != st.bytes[k]) {
                if (t == 0) {
                    st.err = 1;
                    set_status(status, ZIPNN_E_CORRUPT);
                }
            }
        }
        __syncthreads();
        if (st.err) return;
    }
    const uint32_t j = slice * 4 + (t >> 6);
    if (j < NG) {
        uint8_t* out = d.dst + uint64_t(c) * h.E * B;
        const uint8_t* base = DELTA ? d.base + uint64_t(c) * h.E * B : nullptr;
        decode_lane_group<B, G, DELTA, ZGK>(d.src, st, wring, lut, wprefix, h.L, j, W, m, out, base, status,
                                            (h.flags & kFlagExp) != 0);
    }
    __syncthreads();
}

// `descs` == nullptr: decode the single tensor `one`; otherwise the batch
// descs[0..n_desc) whose per-tensor item counts k_plan prefixed.  Every tensor
// of a launch has B-byte words, groups of G, (for DELTA) an XOR base and (for
// ZGK) the header's ZG flag; a header that disagrees is reported as
// ZIPNN_E_FORMAT.  With `work` (batched launches) a workgroup takes its next
// item from that counter, zero at launch, as it finishes one: against items
// handed out grid-stride, the checkpoint decoded 4-9% faster and its deltas
// 7-8%, since workgroups do not run at one speed.  A single-tensor launch
// (work null) stays grid-stride: it needs no counter that launches on other
// streams could share.
// Four waves per SIMD (at most 128 VGPRs) keep enough lanes in flight to
// hide LDS and memory latency; the widest words with the largest groups get
// the registers of two waves instead of spilling (16-byte groups with an
// XOR base count as wide).  (The BF16 ZG delta kernel spills 8 bytes at 128
// VGPRs; at 130 VGPRs and three waves it decoded the ZG delta checkpoint 28%
// slower.)
template <int B, int G, bool DELTA, bool ZGK>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(B * G >= (DELTA ? 16 : 32) ? 2 : 4, 8))) void k_decode(DecDesc one, const DecDesc* __restrict__ descs, int n_desc,
                                                   const uint64_t* __restrict__ item_prefix, int* status,
                                                   unsigned long long* __restrict__ work)
{
    __shared__ uint16_t lut[B][kLutSize];
    __shared__ uint32_t wprefix[B][65];
    // aligned to one ring's size: a ring's words are addressed by OR (huf_take)
    __shared__ __attribute__((aligned(Ring<B>::RW * 4))) uint32_t wring[B * 4 * Ring<B>::RW];
    __shared__ LutTmp T;
    __shared__ ItemState st;
    __shared__ TensorState ts;
    __shared__ uint64_t n_items_sh;
    __shared__ uint64_t item_sh;
    if (descs == nullptr) {
        descs = &one;
        n_desc = 1;
        item_prefix = nullptr;
    }
    auto matches = [&](const TensorState& x) {
        return x.h.B == uint32_t(B) && x.h.g == uint32_t(G) && ((x.h.flags & kFlagDelta) != 0) == DELTA &&
               ((x.h.flags & kFlagZg) != 0) == ZGK;
    };
    if (threadIdx.x == 0) {
        ts.desc = -1;
        if (item_prefix == nullptr) {
            const bool ok = load_tensor(descs[0], 0, ts, status, blockIdx.x == 0);
            if (ok && !matches(ts)) {
                ts.valid = 0;
                if (blockIdx.x == 0) set_status(status, ZIPNN_E_FORMAT);
            }
            n_items_sh = ts.valid ? ts.p.items : 0;
        } else {
            n_items_sh = item_prefix[n_desc];
        }
    }
    __syncthreads();
    const uint64_t n_items = n_items_sh;
    // items from a shared counter when the launch has one, else grid-stride
    auto next_item = [&](uint64_t cur) -> uint64_t {
        if (!work) return cur + gridDim.x;
        if (threadIdx.x == 0) item_sh = atomicAdd(work, 1ull);
        __syncthreads();
        const uint64_t v = item_sh;
        __syncthreads();
        return v;
    };
    const uint64_t first = work ? next_item(0) : uint64_t(blockIdx.x);
    for (uint64_t item = first; item < n_items; item = next_item(item)) {
        if (item_prefix) {
            if (threadIdx.x == 0) {
                // tensor holding this item: last i with prefix[i] <= item
                int lo = 0, hi = n_desc - 1;
                while (lo < hi) {
                    int mid = (lo + hi + 1) >> 1;
                    if (item_prefix[mid] <= item) lo = mid;
                    else hi = mid - 1;
                }
                if (lo != ts.desc) {
                    // the plan gave this tensor items, so its header was valid
                    // when planned; a container changed since then is
                    // reported and its items are skipped
                    const DecDesc& dl = descs[lo];
                    if (load_tensor(dl, lo, ts, status, false) && !matches(ts)) ts.valid = 0;
                    if (!ts.valid) set_status(dl.status ? dl.status : status, ZIPNN_E_FORMAT);
                }
            }
            __syncthreads();
            if (!ts.valid) continue;
        }
        const uint64_t local = item - (item_prefix ? item_prefix[ts.desc] : 0);
        const uint64_t full_items = uint64_t(ts.p.full_chunks) * ts.p.slices_full;
        uint32_t c, slice;
        if (local < full_items) {
            c = ts.p.c0 + uint32_t(local / ts.p.slices_full);
            slice = uint32_t(local % ts.p.slices_full);
        } else {
            c = ts.h.n_chunks - 1;
            slice = uint32_t(local - full_items);
        }
        const DecDesc& d = descs[ts.desc];
        decode_item<B, G, DELTA, ZGK>(d, ts, c, slice, wring, lut, wprefix, T, st, d.status ? d.status : status);
    }
}

// Batched plan: items per tensor -> exclusive prefix (one workgroup).  A
// tensor whose header is invalid or does not match (B, G, DELTA) gets no
// items and is reported.
__global__ __launch_bounds__(kBlock) void k_plan(const DecDesc* __restrict__ descs, int n_desc, DecClass k,
                                                 uint64_t* __restrict__ prefix, int* status,
                                                 unsigned long long* __restrict__ work)
{
    __shared__ TensorState tsv[kBlock];
    __shared__ uint64_t carry;
    if (threadIdx.x == 0) carry = 0;
    if (threadIdx.x == 0 && work) *work = 0;
    __syncthreads();
    for (int b0 = 0; b0 < n_desc; b0 += kBlock) {
        const int i = b0 + threadIdx.x;
        if (i < n_desc && load_tensor(descs[i], i, tsv[threadIdx.x], status, true)) {
            const Header& h = tsv[threadIdx.x].h;
            const DecClass x = dec_class(h);
            if (x.B != k.B || x.G != k.G || x.delta != k.delta || x.zg != k.zg) {
                tsv[threadIdx.x].valid = 0;
                set_status(status, ZIPNN_E_FORMAT);
            }
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            uint64_t run = carry;
            for (int j = 0; j < kBlock && b0 + j < n_desc; j++) {
                prefix[b0 + j] = run;
                run += tsv[j].valid ? tsv[j].p.items : 0;
            }
            carry = run;
            if (b0 + kBlock >= n_desc) prefix[n_desc] = run;
        }
        __syncthreads();
    }
}

__global__ void k_clear(int* p) { *p = 0; }

// Copy the 64-byte header of every container of an arena to `out`.
__global__ void k_gather_headers(const uint8_t* __restrict__ arena, const uint64_t* __restrict__ offs, int n,
                                 uint4* __restrict__ out)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= 4 * n) return;
    out[i] = *(const uint4*)(arena + offs[i >> 2] + 16 * (i & 3));
}

template <int B, int G, bool D, bool Z>
hipError_t launch_k(const DecDesc& one, const DecDesc* descs, int n, const uint64_t* prefix, int* st, int grid,
                    hipStream_t s, unsigned long long* work)
{
    k_decode<B, G, D, Z><<<grid, kBlock, 0, s>>>(one, descs, n, prefix, st, work);
    return hipGetLastError();
}

hipError_t dispatch(const DecClass& k, const DecDesc& one, const DecDesc* descs, int n, const uint64_t* prefix,
                    int* st, int grid, hipStream_t s, unsigned long long* work = nullptr)
{
#define ZIPNN_K(BB, GG)                                                                                       \
    if (k.B == BB && k.G == GG) {                                                                            \
        if (k.zg)                                                                                            \
            return k.delta ? launch_k<BB, GG, true, true>(one, descs, n, prefix, st, grid, s, work)                \
                           : launch_k<BB, GG, false, true>(one, descs, n, prefix, st, grid, s, work);              \
        return k.delta ? launch_k<BB, GG, true, false>(one, descs, n, prefix, st, grid, s, work)                   \
                       : launch_k<BB, GG, false, false>(one, descs, n, prefix, st, grid, s, work);                 \
    }
    ZIPNN_K(1, 2) ZIPNN_K(1, 4) ZIPNN_K(1, 8)
    ZIPNN_K(2, 2) ZIPNN_K(2, 4) ZIPNN_K(2, 8)
    ZIPNN_K(4, 2) ZIPNN_K(4, 4) ZIPNN_K(4, 8)
#undef ZIPNN_K
    return hipErrorInvalidValue;
}

}  // namespace

namespace {
template <int B, int G, bool D, bool Z>
int blocks_per_cu()
{
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_decode<B, G, D, Z>, kBlock, 0) != hipSuccess)
        return 0;
    return per_cu;
}
}  // namespace

// The persistent grid of a kernel class: as many workgroups as fit on the
// device at once for that instantiation (its own registers and LDS).
int decode_grid_size(int device, const DecClass& k)
{
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) != hipSuccess) return 1024;
    int per_cu = 0;
#define ZIPNN_OCC(BB, GG)                                                                                     \
    if (k.B == BB && k.G == GG)                                                                              \
        per_cu = k.zg ? (k.delta ? blocks_per_cu<BB, GG, true, true>() : blocks_per_cu<BB, GG, false, true>()) \
                      : (k.delta ? blocks_per_cu<BB, GG, true, false>() : blocks_per_cu<BB, GG, false, false>());
    ZIPNN_OCC(1, 2) ZIPNN_OCC(1, 4) ZIPNN_OCC(1, 8)
    ZIPNN_OCC(2, 2) ZIPNN_OCC(2, 4) ZIPNN_OCC(2, 8)
    ZIPNN_OCC(4, 2) ZIPNN_OCC(4, 4) ZIPNN_OCC(4, 8)
#undef ZIPNN_OCC
    if (per_cu < 1) per_cu = 2;
    return prop.multiProcessorCount * per_cu;
}

hipError_t launch_decode_one(const Header& h, const DecDesc& one, int* d_status, int grid, hipStream_t s)
{
    return dispatch(dec_class(h), one, nullptr, 1, nullptr, d_status, grid, s);
}

hipError_t launch_decode_batch(const DecClass& k, const DecDesc* d_descs, int n_desc, uint64_t* d_item_prefix,
                               int* d_status, int grid, hipStream_t s)
{
    // the shared item counter sits after the prefix's n_desc + 1 entries
    unsigned long long* work = reinterpret_cast<unsigned long long*>(d_item_prefix + n_desc + 1);
    k_plan<<<1, kBlock, 0, s>>>(d_descs, n_desc, k, d_item_prefix, d_status, work);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    DecDesc none = {};
    return dispatch(k, none, d_descs, n_desc, d_item_prefix, d_status, grid, s, work);
}

hipError_t launch_decode_planned(const DecClass& k, const DecDesc* d_descs, int n_desc, uint64_t* d_item_prefix,
                                 int* d_status, int grid, hipStream_t s)
{
    DecDesc none = {};
    unsigned long long* work = reinterpret_cast<unsigned long long*>(d_item_prefix + n_desc + 1);
    return dispatch(k, none, d_descs, n_desc, d_item_prefix, d_status, grid, s, work);
}

hipError_t launch_gather_headers(const uint8_t* arena, const uint64_t* d_offs, int n, void* d_out, hipStream_t s)
{
    k_gather_headers<<<(4 * n + 255) / 256, 256, 0, s>>>(arena, d_offs, n, (uint4*)d_out);
    return hipGetLastError();
}

hipError_t launch_clear_status(int* d_status, hipStream_t s)
{
    k_clear<<<1, 1, 0, s>>>(d_status);
    return hipGetLastError();
}

}  // namespace zipnn
