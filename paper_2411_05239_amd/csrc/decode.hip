// Decode kernels of the gfx950 ZipNN codec.
//
// Work item = (tensor, chunk, slice of up to 256 sub-streams).  Chunks are
// independent given the map (paper §V-A "Metadata and parallelism"), and
// inside a chunk the W interleaved sub-streams of every Huffman-coded byte
// group are independent too, so one workgroup of 256 threads decodes one
// slice: thread t owns sub-stream w = 256*slice + t of EVERY stream of the
// chunk.  Because all streams of a chunk share the same (m, S, g), sub-stream
// w of every stream covers the same element positions (groups q = w, w+W,
// ...), so a thread merges the B byte groups back into words in registers
// (the inverse of byte grouping, paper §III-A/§III-B), applies the XOR delta
// (paper §IV-B) and writes g whole words with one vector store; a wave writes
// 64*g*B contiguous bytes per step.
//
// Per item:
//   1. the B map entries are read and checked (mode, sizes, the exact
//      chunk-major 16-byte aligned placement) into LDS;
//   2. each Huffman table (128 B of 4-bit lengths) is checked (Kraft sum
//      exactly 2^L, >= 2 codes, lengths <= L) and expanded into a 2^L-entry
//      LDS lookup table {symbol, length} indexed by the next L stream bits;
//   3. the u16 sub-stream lengths are scanned to find each thread's start bit
//      and checked against the payload size;
//   4. the hot loop: per group, every HUF stream peeks L bits, looks up
//      (symbol, length) in LDS and consumes; RAW streams load g bytes; RLE
//      streams splat their value; words are assembled and stored;
//   5. every sub-stream must consume exactly its stored bit length.
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
    uint32_t bitbase[4];   // first bit of this slice's first sub-stream
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
    uint32_t slices_full;  // slices per full chunk
    uint32_t slices_last;
    uint64_t items;
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

// Exclusive scan over the 256 threads of the block; *total gets the sum.
__device__ inline uint32_t block_excl_scan(uint32_t v, uint32_t* red, uint32_t* total)
{
    uint32_t inc = wave_incl_scan(v);
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    if (lane == 63) red[wv] = inc;
    __syncthreads();
    uint32_t pre = 0, tot = 0;
#pragma unroll
    for (int i = 0; i < 4; i++) {
        uint32_t s = red[i];
        pre += i < wv ? s : 0;
        tot += s;
    }
    __syncthreads();
    *total = tot;
    return pre + inc - v;
}

__device__ inline uint32_t block_sum(uint32_t v, uint32_t* red)
{
    uint32_t t;
    block_excl_scan(v, red, &t);
    return t;
}

// Expand a 128-byte nibble table into the LSB-first lookup table `lut`
// (entry = symbol | length << 8 for every L-bit window).  Returns false (in
// every thread) when the lengths are not a complete prefix code.
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
        T.entry[pos] = uint16_t(t | (l << 8));
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

// Bit reader over one sub-stream: 64-bit window, refilled one dword at a
// time; loads past the payload are clamped to its last dword (those bits are
// never consumed by a well-formed sub-stream).
struct BitReader {
    const uint32_t* bs;
    uint32_t last;
    uint32_t idx;
    uint32_t cnt;
    uint64_t buf;
    uint32_t start;

    __device__ inline void init(const uint32_t* base, uint32_t last_dw, uint32_t bit)
    {
        bs = base;
        last = last_dw;
        start = bit;
        idx = bit >> 5;
        uint32_t sh = bit & 31;
        buf = uint64_t(bs[min(idx, last)] >> sh);
        cnt = 32 - sh;
        idx++;
        refill();
    }
    __device__ inline void refill()
    {
        if (cnt <= 32) {
            buf |= uint64_t(bs[min(idx, last)]) << cnt;
            cnt += 32;
            idx++;
        }
    }
    __device__ inline uint32_t get(const uint16_t* lut, uint32_t mask)
    {
        uint32_t e = lut[uint32_t(buf) & mask];
        uint32_t l = e >> 8;
        buf >>= l;
        cnt -= l;
        return e & 0xFF;
    }
    __device__ inline uint32_t consumed() const { return idx * 32u - cnt - start; }
};

template <int G>
struct RawLoad;
template <>
struct RawLoad<1> {
    static __device__ inline void run(const uint8_t* p, uint32_t* o) { o[0] = p[0]; }
};
template <>
struct RawLoad<2> {
    static __device__ inline void run(const uint8_t* p, uint32_t* o) { o[0] = *(const uint16_t*)p; }
};
template <>
struct RawLoad<4> {
    static __device__ inline void run(const uint8_t* p, uint32_t* o) { o[0] = *(const uint32_t*)p; }
};
template <>
struct RawLoad<8> {
    static __device__ inline void run(const uint8_t* p, uint32_t* o)
    {
        uint2 v = *(const uint2*)p;
        o[0] = v.x;
        o[1] = v.y;
    }
};

template <int NB>
struct Store;
template <>
struct Store<1> {
    static __device__ inline void run(uint8_t* d, const uint32_t* w) { d[0] = uint8_t(w[0]); }
    static __device__ inline void xor_base(const uint8_t* b, uint32_t* w) { w[0] ^= b[0]; }
};
template <>
struct Store<2> {
    static __device__ inline void run(uint8_t* d, const uint32_t* w) { *(uint16_t*)d = uint16_t(w[0]); }
    static __device__ inline void xor_base(const uint8_t* b, uint32_t* w) { w[0] ^= *(const uint16_t*)b; }
};
template <>
struct Store<4> {
    static __device__ inline void run(uint8_t* d, const uint32_t* w) { *(uint32_t*)d = w[0]; }
    static __device__ inline void xor_base(const uint8_t* b, uint32_t* w) { w[0] ^= *(const uint32_t*)b; }
};
template <>
struct Store<8> {
    static __device__ inline void run(uint8_t* d, const uint32_t* w) { *(uint2*)d = make_uint2(w[0], w[1]); }
    static __device__ inline void xor_base(const uint8_t* b, uint32_t* w)
    {
        uint2 v = *(const uint2*)b;
        w[0] ^= v.x;
        w[1] ^= v.y;
    }
};
template <>
struct Store<16> {
    static __device__ inline void run(uint8_t* d, const uint32_t* w) { *(uint4*)d = make_uint4(w[0], w[1], w[2], w[3]); }
    static __device__ inline void xor_base(const uint8_t* b, uint32_t* w)
    {
        uint4 v = *(const uint4*)b;
        w[0] ^= v.x;
        w[1] ^= v.y;
        w[2] ^= v.z;
        w[3] ^= v.w;
    }
};
template <>
struct Store<32> {
    static __device__ inline void run(uint8_t* d, const uint32_t* w)
    {
        *(uint4*)d = make_uint4(w[0], w[1], w[2], w[3]);
        *(uint4*)(d + 16) = make_uint4(w[4], w[5], w[6], w[7]);
    }
    static __device__ inline void xor_base(const uint8_t* b, uint32_t* w)
    {
        Store<16>::xor_base(b, w);
        Store<16>::xor_base(b + 16, w + 4);
    }
};

template <int B>
__device__ inline uint32_t stream_byte(const uint32_t (*pk)[2], int k, int i)
{
    return (pk[k][i >> 2] >> (8 * (i & 3))) & 0xFFu;
}

// Decode the groups of sub-stream w of one chunk and store merged words.
template <int B, int G>
__device__ void decode_substream(const uint8_t* __restrict__ src, const ItemState& st,
                                 const uint16_t (*lut)[kLutSize], uint32_t L, uint32_t w, uint32_t W, uint32_t m,
                                 const uint32_t* bitstart, uint8_t* __restrict__ out,
                                 const uint8_t* __restrict__ base, int* status)
{
    constexpr int NBYTES = B * G;
    constexpr int NW = NBYTES >= 4 ? NBYTES / 4 : 1;
    const uint32_t mask = (1u << L) - 1;
    int mode[B];
    uint32_t rlev[B];
    const uint8_t* pay[B];
    BitReader br[B];
#pragma unroll
    for (int k = 0; k < B; k++) {
        mode[k] = __builtin_amdgcn_readfirstlane(st.mode[k]);
        rlev[k] = st.rle[k] * 0x01010101u;
        pay[k] = src + st.pay[k];
        if (mode[k] == kModeHuf) {
            const uint32_t W_ = W;
            const uint32_t head = huf_head(W_);
            const uint32_t* bs = (const uint32_t*)(pay[k] + head);
            const uint32_t ext = uint32_t(align16(st.bytes[k])) - head;   // bytes of bitstream area
            br[k].init(bs, ext / 4 - 1, bitstart[k]);
        }
    }
    const uint32_t Gfull = m / G;
    for (uint32_t q = w; q < Gfull; q += W) {
        const uint32_t e = q * G;
        uint32_t pk[B][2];
#pragma unroll
        for (int k = 0; k < B; k++) {
            pk[k][0] = pk[k][1] = 0;
            if (mode[k] == kModeRaw) {
                RawLoad<G>::run(pay[k] + e, pk[k]);
            } else if (mode[k] == kModeRle) {
                pk[k][0] = pk[k][1] = rlev[k];
            } else {
#pragma unroll
                for (int i = 0; i < G; i++) {
                    if ((i & 1) == 0) br[k].refill();
                    pk[k][i >> 2] |= br[k].get(lut[k], mask) << (8 * (i & 3));
                }
            }
        }
        uint32_t ow[NW];
#pragma unroll
        for (int x = 0; x < NW; x++) ow[x] = 0;
#pragma unroll
        for (int j = 0; j < NBYTES; j++) {
            const int i = j / B, b = j % B;
            ow[j >> 2] |= stream_byte<B>(pk, B - 1 - b, i) << (8 * (j & 3));
        }
        uint8_t* d = out + uint64_t(e) * B;
        if (base) Store<NBYTES>::xor_base(base + uint64_t(e) * B, ow);
        Store<NBYTES>::run(d, ow);
    }
    // a partial last group (only in the last chunk of a tensor)
    const uint32_t rem = m - Gfull * G;
    if (rem && (Gfull % W) == w) {
        const uint32_t e = Gfull * G;
        uint32_t sy[B][G];
#pragma unroll
        for (int k = 0; k < B; k++) {
#pragma unroll
            for (int i = 0; i < G; i++) {
                sy[k][i] = 0;
                if (uint32_t(i) < rem) {
                    if (mode[k] == kModeRaw) sy[k][i] = pay[k][e + i];
                    else if (mode[k] == kModeRle) sy[k][i] = rlev[k] & 0xFF;
                    else {
                        br[k].refill();
                        sy[k][i] = br[k].get(lut[k], mask);
                    }
                }
            }
        }
        for (uint32_t i = 0; i < rem; i++) {
#pragma unroll
            for (int b = 0; b < B; b++) {
                uint8_t v = uint8_t(sy[B - 1 - b][0]);
#pragma unroll
                for (int ii = 0; ii < G; ii++)
                    if (uint32_t(ii) == i) v = uint8_t(sy[B - 1 - b][ii]);
                uint64_t o = uint64_t(e + i) * B + b;
                out[o] = base ? uint8_t(v ^ base[o]) : v;
            }
        }
    }
#pragma unroll
    for (int k = 0; k < B; k++) {
        if (mode[k] == kModeHuf) {
            // the stored length of this sub-stream
            const uint16_t* lens = (const uint16_t*)(pay[k] + 128);
            if (br[k].consumed() != lens[w]) set_status(status, ZIPNN_E_CORRUPT);
        }
    }
}

__device__ bool load_tensor(const DecDesc& d, int di, TensorState& ts, int* status, bool report)
{
    // every thread reads the header (64 B, served from cache after the first)
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
    ts.items = 0;
    if (rc != ZIPNN_OK) {
        if (report && threadIdx.x == 0) set_status(status, rc);
        return false;
    }
    const uint32_t Wf = (ts.h.E + ts.h.S - 1) / ts.h.S;
    ts.slices_full = (Wf + kBlock - 1) / kBlock;
    if (ts.h.n_chunks == 0) return true;
    const uint64_t m_last = ts.h.n - uint64_t(ts.h.n_chunks - 1) * ts.h.E;
    const uint32_t Wl = uint32_t((m_last + ts.h.S - 1) / ts.h.S);
    ts.slices_last = (Wl + kBlock - 1) / kBlock;
    ts.items = uint64_t(ts.h.n_chunks - 1) * ts.slices_full + ts.slices_last;
    return true;
}

__device__ void decode_item(const DecDesc& d, const TensorState& ts, uint32_t c, uint32_t slice,
                            uint16_t (*lut)[kLutSize], LutTmp& T, ItemState& st, int* status)
{
    const Header& h = ts.h;
    const int t = threadIdx.x;
    const uint32_t B = h.B;
    const uint32_t m = uint32_t(min(uint64_t(h.E), h.n - uint64_t(c) * h.E));
    const uint32_t W = (m + h.S - 1) / h.S;
    if (t == 0) st.err = 0;
    __syncthreads();
    if (t < int(B)) {
        const uint64_t e = uint64_t(c) * B + t;
        const uint4 ent = *(const uint4*)(d.src + 64 + 16 * e);
        const uint64_t off = uint64_t(ent.x) | (uint64_t(ent.y) << 32);
        const uint32_t bytes = ent.z;
        const uint32_t mode = ent.w & 0xFF, rle = (ent.w >> 8) & 0xFF;
        int err = 0;
        if ((ent.w >> 16) != 0 || mode > 2) err = 1;
        if (mode == kModeRaw && (bytes != m || rle)) err = 1;
        if (mode == kModeRle && bytes != 0) err = 1;
        if (mode == kModeHuf && (bytes < huf_head(W) || rle)) err = 1;
        if (off & 15) err = 1;
        // the exact placement: this entry starts where its predecessor ends
        uint64_t expect = 0;
        if (e > 0) {
            const uint4 pe = *(const uint4*)(d.src + 64 + 16 * (e - 1));
            const uint64_t poff = uint64_t(pe.x) | (uint64_t(pe.y) << 32);
            expect = poff + align16(pe.z);
        }
        if (off != expect) err = 1;
        if (h.payload_base + off + bytes > h.total) err = 1;
        if (e + 1 == uint64_t(h.n_chunks) * B && h.payload_base + off + align16(bytes) != h.total) err = 1;
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
    uint32_t bitstart[4] = {0, 0, 0, 0};
    const uint32_t w = slice * kBlock + t;
    for (uint32_t k = 0; k < B; k++) {
        if (st.mode[k] != kModeHuf) continue;
        const uint8_t* p = d.src + st.pay[k];
        if (!build_lut(p, h.L, lut[k], T)) {
            if (t == 0) {
                st.err = 1;
                set_status(status, ZIPNN_E_CORRUPT);
            }
            __syncthreads();
            return;
        }
        const uint16_t* lens = (const uint16_t*)(p + 128);
        uint32_t pre = 0, tot = 0, mine = 0;
        for (uint32_t v = t; v < W; v += kBlock) {
            uint32_t l = lens[v];
            tot += l;
            if (v < slice * kBlock) pre += l;
            if (v == w) mine = l;
        }
        tot = block_sum(tot, T.red);
        pre = block_sum(pre, T.red);
        uint32_t dummy;
        const uint32_t off = block_excl_scan(mine, T.red, &dummy);
        bitstart[k] = pre + off;
        // every symbol takes at least one bit, and the payload must end
        // exactly where the bitstream does
        if (tot < m || st.bytes[k] != huf_head(W) + (tot + 7) / 8) {
            if (t == 0) {
                st.err = 1;
                set_status(status, ZIPNN_E_CORRUPT);
            }
        }
        __syncthreads();
        if (st.err) return;
    }
    if (w < W) {
        uint8_t* out = d.dst + uint64_t(c) * h.E * B;
        const uint8_t* base = d.base ? d.base + uint64_t(c) * h.E * B : nullptr;
        const uint16_t(*cl)[kLutSize] = lut;
        switch (B * 16 + h.g) {
#define ZIPNN_CASE(BB, GG)                                                                          \
    case BB * 16 + GG:                                                                             \
        decode_substream<BB, GG>(d.src, st, cl, h.L, w, W, m, bitstart, out, base, status);        \
        break;
            ZIPNN_CASE(1, 1)
            ZIPNN_CASE(1, 2)
            ZIPNN_CASE(1, 4)
            ZIPNN_CASE(1, 8)
            ZIPNN_CASE(2, 1)
            ZIPNN_CASE(2, 2)
            ZIPNN_CASE(2, 4)
            ZIPNN_CASE(2, 8)
            ZIPNN_CASE(4, 1)
            ZIPNN_CASE(4, 2)
            ZIPNN_CASE(4, 4)
            ZIPNN_CASE(4, 8)
#undef ZIPNN_CASE
        default:
            set_status(status, ZIPNN_E_FORMAT);
        }
    }
    __syncthreads();
}

// `descs` == nullptr: decode the single tensor `one` (its header parsed on
// the device, no host round trip); otherwise the batch descs[0..n_desc) whose
// per-tensor item counts were prefixed by k_plan.
__global__ __launch_bounds__(kBlock) void k_decode(DecDesc one, const DecDesc* __restrict__ descs, int n_desc,
                                                   const uint64_t* __restrict__ item_prefix, int* status)
{
    if (descs == nullptr) {
        descs = &one;
        n_desc = 1;
        item_prefix = nullptr;
    }
    __shared__ uint16_t lut[4][kLutSize];
    __shared__ LutTmp T;
    __shared__ ItemState st;
    __shared__ TensorState ts;
    __shared__ uint64_t n_items_sh;
    if (threadIdx.x == 0) {
        ts.desc = -1;
        if (item_prefix == nullptr) {
            load_tensor(descs[0], 0, ts, status, blockIdx.x == 0);
            n_items_sh = ts.valid ? ts.items : 0;
        } else {
            n_items_sh = item_prefix[n_desc];
        }
    }
    __syncthreads();
    const uint64_t n_items = n_items_sh;
    for (uint64_t item = blockIdx.x; item < n_items; item += gridDim.x) {
        if (item_prefix) {
            if (threadIdx.x == 0) {
                // tensor holding this item: last i with prefix[i] <= item
                int lo = 0, hi = n_desc - 1;
                while (lo < hi) {
                    int mid = (lo + hi + 1) >> 1;
                    if (item_prefix[mid] <= item) lo = mid;
                    else hi = mid - 1;
                }
                if (lo != ts.desc) load_tensor(descs[lo], lo, ts, status, false);
            }
            __syncthreads();
        }
        const uint64_t local = item - (item_prefix ? item_prefix[ts.desc] : 0);
        const uint32_t full_items = (ts.h.n_chunks - 1) * ts.slices_full;
        uint32_t c, slice;
        if (local < full_items) {
            c = uint32_t(local / ts.slices_full);
            slice = uint32_t(local % ts.slices_full);
        } else {
            c = ts.h.n_chunks - 1;
            slice = uint32_t(local - full_items);
        }
        decode_item(descs[ts.desc], ts, c, slice, lut, T, st, status);
    }
}

// Batched plan: items per tensor -> exclusive prefix (one workgroup).
__global__ __launch_bounds__(kBlock) void k_plan(const DecDesc* __restrict__ descs, int n_desc,
                                                 uint64_t* __restrict__ prefix, int* status)
{
    __shared__ TensorState tsv[kBlock];
    __shared__ uint64_t carry;
    if (threadIdx.x == 0) carry = 0;
    __syncthreads();
    for (int base = 0; base < n_desc; base += kBlock) {
        const int i = base + threadIdx.x;
        uint64_t items = 0;
        if (i < n_desc && load_tensor(descs[i], i, tsv[threadIdx.x], status, true)) items = tsv[threadIdx.x].items;
        __syncthreads();
        if (threadIdx.x == 0) {
            uint64_t run = carry;
            for (int j = 0; j < kBlock && base + j < n_desc; j++) {
                prefix[base + j] = run;
                run += tsv[j].valid ? tsv[j].items : 0;
            }
            carry = run;
            if (base + kBlock >= n_desc) prefix[n_desc] = run;
        }
        __syncthreads();
    }
}

}  // namespace

int decode_grid_size(int device)
{
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) != hipSuccess) return 1024;
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_decode, kBlock, 0) != hipSuccess || per_cu < 1)
        per_cu = 4;
    return prop.multiProcessorCount * per_cu;
}

hipError_t launch_decode_one(const DecDesc& one, int* d_status, int grid, hipStream_t s)
{
    k_decode<<<grid, kBlock, 0, s>>>(one, nullptr, 1, nullptr, d_status);
    return hipGetLastError();
}

hipError_t launch_decode_batch(const DecDesc* d_descs, int n_desc, uint64_t* d_item_prefix, int* d_status, int grid,
                               hipStream_t s)
{
    k_plan<<<1, kBlock, 0, s>>>(d_descs, n_desc, d_item_prefix, d_status);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    DecDesc none = {};
    k_decode<<<grid, kBlock, 0, s>>>(none, d_descs, n_desc, d_item_prefix, d_status);
    return hipGetLastError();
}

__global__ void k_clear(int* p) { *p = 0; }

hipError_t launch_clear_status(int* d_status, hipStream_t s)
{
    k_clear<<<1, 1, 0, s>>>(d_status);
    return hipGetLastError();
}

}  // namespace zipnn
