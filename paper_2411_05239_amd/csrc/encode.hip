// Encode kernels of the gfx950 ZipNN codec.
//
//   k_analyze  one workgroup per chunk: reads the chunk once (16-byte loads,
//              XOR with the base for a delta, paper §IV-B), splits every word
//              into its B byte groups (paper §III-A/§III-B) and histograms
//              each group in LDS; then wave k builds the code of group k:
//              optimal lengths <= L by package-merge (Larmore & Hirschberg,
//              computed with parallel ranks, see build_code), canonical codes
//              (RFC 1951 §3.2.2), the coded size and the per-byte-group method
//              (paper §V-A): RAW / RLE for a single value (paper §III-B) /
//              HUF only if smaller than raw under AUTO.
//   k_place    one workgroup per tensor: exclusive scan of the 16-byte aligned
//              payload sizes in chunk-major order -> map entries and header
//              (the map that enables parallel decode, paper §V-A).
//   k_pack     one workgroup per chunk: thread t owns sub-streams t, t+256, ...
//              pass A sums code lengths per sub-stream, a block scan gives bit
//              offsets, pass B writes the codes (bits shared with a neighbour
//              sub-stream go through atomicOr on pre-zeroed dwords) and the
//              RAW groups; every byte of the payload extent, padding included,
//              is written.
#include "zipnn_internal.h"

namespace zipnn {
namespace {

constexpr int kWaves = kBlock / 64;

struct PmWave {                 // package-merge workspace of one wave
    uint32_t leafw[256];        // leaf weights, ascending (f, symbol)
    uint16_t leafsym[256];
    uint32_t pk[256];           // package weights of the current level
    uint32_t cur[512];          // current list weights
    uint16_t pos[kMaxL][256];   // position of leaf i in the list of each level
    uint32_t key[256];
    uint8_t len[256];           // code length per symbol
    uint32_t cnt[16];
};

union AnalyzeLds {
    uint32_t hist[kWaves][4][256];   // per-wave sub-histograms (phase 1)
    PmWave pm[kWaves];               // per-wave code construction (phase 2)
};

__device__ inline uint32_t wave_sum(uint32_t v)
{
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d, 64);
    return v;
}

// number of items of a sorted u32 array a[0..n) that are < x (strict) or <= x
__device__ inline uint32_t count_lt(const uint32_t* a, uint32_t n, uint32_t x)
{
    uint32_t lo = 0, hi = n;
    while (lo < hi) {
        uint32_t mid = (lo + hi) >> 1;
        if (a[mid] < x) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}
__device__ inline uint32_t count_le(const uint32_t* a, uint32_t n, uint32_t x)
{
    uint32_t lo = 0, hi = n;
    while (lo < hi) {
        uint32_t mid = (lo + hi) >> 1;
        if (a[mid] <= x) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

// Build the code of one byte group with one wave.  f[] is the histogram.
// Writes codes[256] (canonical code | length << 16) and the entry.
//
// Package-merge with lists made of leaves and packages: list 0 = the leaves
// sorted by (f, symbol); list d = the leaves merged with the packages of
// consecutive pairs of list d-1, a leaf before a package of equal weight.
// Merging two sorted sequences is done by ranks: leaf i lands at
// i + #{packages lighter than it}, package j at j + #{leaves not heavier}.
// The 2n'-2 first items of the top list are selected; the packages among the
// first m items of a list select the first 2*(their count) items of the list
// below; leaf i is selected at a level iff i < (leaves among the selected
// items), so its length is the number of such levels.
__device__ void build_code(const uint32_t* f, uint32_t m, uint32_t W, uint32_t L, int policy, PmWave& P,
                           CodeWord* codes, EncEntry* entry)
{
    const int lane = threadIdx.x & 63;
    uint32_t fv[4];
    uint32_t d = 0;
#pragma unroll
    for (int r = 0; r < 4; r++) {
        fv[r] = f[lane + 64 * r];
        d += __popcll(__ballot(fv[r] > 0));
    }
    for (int r = 0; r < 4; r++) codes[lane + 64 * r] = 0;
    if (policy == ZIPNN_RAW || d <= 1) {
        if (lane == 0) {
            EncEntry e;
            e.pad = 0;
            if (policy != ZIPNN_RAW && d == 1) {
                uint32_t v = 0;
                for (int s = 0; s < 256; s++)
                    if (f[s]) v = s;
                e.mode = kModeRle;
                e.rle = uint8_t(v);
                e.bytes = 0;
            } else {
                e.mode = kModeRaw;
                e.rle = 0;
                e.bytes = m;
            }
            *entry = e;
        }
        return;
    }
    // sort the leaves by key = f << 8 | symbol (f < 2^24 since m <= 2^22)
#pragma unroll
    for (int r = 0; r < 4; r++) P.key[lane + 64 * r] = fv[r] ? ((fv[r] << 8) | uint32_t(lane + 64 * r)) : 0xFFFFFFFFu;
    __builtin_amdgcn_wave_barrier();
#pragma unroll
    for (int r = 0; r < 4; r++) {
        if (fv[r]) {
            const uint32_t k = P.key[lane + 64 * r];
            uint32_t rank = 0;
            for (int s = 0; s < 256; s++) rank += P.key[s] < k;
            P.leafw[rank] = fv[r];
            P.leafsym[rank] = uint16_t(lane + 64 * r);
        }
    }
    __builtin_amdgcn_wave_barrier();
    const uint32_t n = d;
    // level 0
    for (uint32_t i = lane; i < n; i += 64) {
        P.cur[i] = P.leafw[i];
        P.pos[0][i] = uint16_t(i);
    }
    uint32_t curlen = n;
    __builtin_amdgcn_wave_barrier();
    for (uint32_t lev = 1; lev < L; lev++) {
        const uint32_t npk = curlen / 2;
        for (uint32_t j = lane; j < npk; j += 64) P.pk[j] = P.cur[2 * j] + P.cur[2 * j + 1];
        __builtin_amdgcn_wave_barrier();
        for (uint32_t i = lane; i < n; i += 64) {
            uint32_t p = i + count_lt(P.pk, npk, P.leafw[i]);
            P.pos[lev][i] = uint16_t(p);
            P.cur[p] = P.leafw[i];
        }
        for (uint32_t j = lane; j < npk; j += 64) {
            uint32_t p = j + count_le(P.leafw, n, P.pk[j]);
            P.cur[p] = P.pk[j];
        }
        curlen = n + npk;
        __builtin_amdgcn_wave_barrier();
    }
    // selection, top level first
    uint32_t lens_local[4] = {0, 0, 0, 0};   // for leaves i = lane + 64 r
    uint32_t sel = 2 * n - 2;
    for (int lev = int(L) - 1; lev >= 0; lev--) {
        uint32_t c = 0;
#pragma unroll
        for (int r = 0; r < 4; r++) {
            uint32_t i = lane + 64 * r;
            c += (i < n && P.pos[lev][i] < sel) ? 1u : 0u;
        }
        c = wave_sum(c);
#pragma unroll
        for (int r = 0; r < 4; r++) lens_local[r] += (uint32_t(lane + 64 * r) < c) ? 1u : 0u;
        sel = 2 * (sel - c);
    }
    // lengths per symbol, cost T
    uint32_t T = 0;
    for (int r = 0; r < 4; r++) P.len[lane + 64 * r] = 0;
    __builtin_amdgcn_wave_barrier();
#pragma unroll
    for (int r = 0; r < 4; r++) {
        uint32_t i = lane + 64 * r;
        if (i < n) {
            P.len[P.leafsym[i]] = uint8_t(lens_local[r]);
            T += P.leafw[i] * lens_local[r];
        }
    }
    T = wave_sum(T);
    const uint32_t size_huf = huf_head(W) + (T + 7) / 8;
    if (policy == ZIPNN_AUTO && size_huf >= m) {
        if (lane == 0) {
            EncEntry e;
            e.pad = 0;
            e.mode = kModeRaw;
            e.rle = 0;
            e.bytes = m;
            *entry = e;
        }
        return;
    }
    __builtin_amdgcn_wave_barrier();
    // canonical codes: first code of each length, then rank within a length
    // in increasing symbol order
    uint32_t l4[4];
#pragma unroll
    for (int r = 0; r < 4; r++) l4[r] = P.len[lane + 64 * r];
    if (lane < 16) P.cnt[lane] = 0;
    __builtin_amdgcn_wave_barrier();
    const uint64_t lt_mask = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    uint32_t rank4[4] = {0, 0, 0, 0};
    for (uint32_t len = 1; len <= L; len++) {
        uint32_t run = 0;
#pragma unroll
        for (int r = 0; r < 4; r++) {
            uint64_t msk = __ballot(l4[r] == len);
            if (l4[r] == len) rank4[r] = run + __popcll(msk & lt_mask);
            run += __popcll(msk);
        }
        if (lane == 0) P.cnt[len] = run;
    }
    __builtin_amdgcn_wave_barrier();
    {
        uint32_t code = 0, prev = 0;
        for (uint32_t len = 1; len <= L; len++) {
            code = (code + prev) << 1;
            prev = P.cnt[len];
#pragma unroll
            for (int r = 0; r < 4; r++)
                if (l4[r] == len) rank4[r] += code;
        }
    }
#pragma unroll
    for (int r = 0; r < 4; r++) codes[lane + 64 * r] = l4[r] ? (rank4[r] | (l4[r] << 16)) : 0u;
    if (lane == 0) {
        EncEntry e;
        e.pad = 0;
        e.mode = kModeHuf;
        e.rle = 0;
        e.bytes = size_huf;
        *entry = e;
    }
}

__device__ inline int find_desc(const uint32_t* prefix, int n_desc, uint32_t g)
{
    int lo = 0, hi = n_desc - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (prefix[mid] <= g) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

__global__ __launch_bounds__(kBlock) void k_analyze(EncDesc one, const EncDesc* __restrict__ descs, int n_desc,
                                                    const uint32_t* __restrict__ chunk_prefix, uint32_t total_chunks,
                                                    EncParams p, EncEntry* __restrict__ entries,
                                                    CodeWord* __restrict__ codes)
{
    __shared__ AnalyzeLds S;
    __shared__ uint32_t hist[4][256];
    const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
    const uint32_t B = p.B;
    for (uint32_t gc = blockIdx.x; gc < total_chunks; gc += gridDim.x) {
        const int di = descs ? find_desc(chunk_prefix, n_desc, gc) : 0;
        const EncDesc d = descs ? descs[di] : one;
        const uint32_t c = gc - (descs ? chunk_prefix[di] : 0);
        const uint32_t E = p.chunk / B;
        const uint64_t e0 = uint64_t(c) * E;
        const uint32_t m = uint32_t(min(uint64_t(E), d.n - e0));
        for (uint32_t i = t; i < kWaves * 4 * 256; i += kBlock) (&S.hist[0][0][0])[i] = 0;
        __syncthreads();
        const uint8_t* src = d.src + e0 * B;
        const uint8_t* base = d.base ? d.base + e0 * B : nullptr;
        const uint32_t nbytes = m * B;
        uint32_t(*h)[256] = S.hist[wv];
        // 16-byte vectors; the element boundary is aligned since 16 % B == 0
        const uint32_t nvec = nbytes / 16;
        for (uint32_t v = t; v < nvec; v += kBlock) {
            uint4 x = ((const uint4*)src)[v];
            if (base) {
                uint4 y = ((const uint4*)base)[v];
                x.x ^= y.x;
                x.y ^= y.y;
                x.z ^= y.z;
                x.w ^= y.w;
            }
            const uint32_t wds[4] = {x.x, x.y, x.z, x.w};
#pragma unroll
            for (int j = 0; j < 16; j++) {
                const uint32_t byte = (wds[j >> 2] >> (8 * (j & 3))) & 0xFF;
                const int k = int(B) - 1 - (j % int(B));   // byte j%B of a word -> stream B-1-j%B
                atomicAdd(&h[k][byte], 1u);
            }
        }
        for (uint32_t b = nvec * 16 + t; b < nbytes; b += kBlock) {
            uint32_t byte = src[b] ^ (base ? base[b] : 0);
            atomicAdd(&h[B - 1 - (b % B)][byte], 1u);
        }
        __syncthreads();
        for (uint32_t i = t; i < 4 * 256; i += kBlock) {
            const uint32_t k = i >> 8, s = i & 255;
            hist[k][s] = S.hist[0][k][s] + S.hist[1][k][s] + S.hist[2][k][s] + S.hist[3][k][s];
        }
        __syncthreads();
        if (uint32_t(wv) < B) {
            const uint32_t W = (m + p.S - 1) / p.S;
            const uint64_t ei = uint64_t(gc) * B + wv;
            build_code(hist[wv], m, W, p.L, p.policy[wv], S.pm[wv], codes + ei * 256, entries + ei);
        }
        __syncthreads();
        (void)lane;
    }
}

// One workgroup per tensor: offsets of its entries and its header + map.
__global__ __launch_bounds__(kBlock) void k_place(EncDesc one, const EncDesc* __restrict__ descs, EncParams p,
                                                  const EncEntry* __restrict__ entries, uint64_t* __restrict__ offsets,
                                                  uint64_t* __restrict__ totals)
{
    __shared__ uint64_t red[kWaves];
    __shared__ uint64_t carry;
    const EncDesc d = descs ? descs[blockIdx.x] : one;
    const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
    const uint32_t B = p.B;
    const uint64_t ne = uint64_t(d.n_chunks) * B;
    const uint64_t e_first = uint64_t(d.chunk0) * B;
    const uint64_t payload_base = 64 + 16 * ne;
    if (t == 0) carry = 0;
    __syncthreads();
    for (uint64_t b0 = 0; b0 < ne; b0 += kBlock) {
        const uint64_t e = b0 + t;
        EncEntry en = {0, 0, 0, 0};
        if (e < ne) en = entries[e_first + e];
        uint64_t sz = align16(en.bytes);
        // inclusive wave scan
        uint64_t inc = sz;
#pragma unroll
        for (int dd = 1; dd < 64; dd <<= 1) {
            uint64_t o = __shfl_up(inc, dd, 64);
            if (lane >= dd) inc += o;
        }
        if (lane == 63) red[wv] = inc;
        __syncthreads();
        uint64_t pre = carry;
        for (int i = 0; i < wv; i++) pre += red[i];
        const uint64_t off = pre + inc - sz;
        if (e < ne) {
            offsets[e_first + e] = off;
            uint4 ent;
            ent.x = uint32_t(off);
            ent.y = uint32_t(off >> 32);
            ent.z = en.bytes;
            ent.w = uint32_t(en.mode) | (uint32_t(en.rle) << 8);
            *(uint4*)(d.dst + 64 + 16 * e) = ent;
        }
        __syncthreads();
        if (t == kBlock - 1) carry = pre + inc;
        __syncthreads();
    }
    if (t == 0) {
        const uint64_t total = payload_base + carry;
        totals[blockIdx.x] = total;
        uint32_t h[16];
        h[0] = 0x314E4E5Au;
        h[1] = 1u | (p.dtype << 16) | (B << 24);
        h[2] = uint32_t(d.n);
        h[3] = uint32_t(d.n >> 32);
        h[4] = p.chunk;
        h[5] = p.S | (p.g << 16) | (p.L << 24);
        h[6] = d.base ? kFlagDelta : 0u;
        h[7] = d.n_chunks;
        h[8] = uint32_t(total);
        h[9] = uint32_t(total >> 32);
        h[10] = 0;
        for (uint32_t k = 0; k < B; k++) h[10] |= uint32_t(p.policy[k]) << (8 * k);
        for (int i = 11; i < 16; i++) h[i] = 0;
        uint4* o = (uint4*)d.dst;
        for (int i = 0; i < 4; i++) o[i] = make_uint4(h[4 * i], h[4 * i + 1], h[4 * i + 2], h[4 * i + 3]);
    }
}

// Load NB bytes (NB in {1,2,4,8,16,32}) from p into 32-bit words.
template <int NB>
__device__ inline void loadNB(const uint8_t* p, uint32_t* w)
{
    if constexpr (NB == 1) w[0] = p[0];
    else if constexpr (NB == 2) w[0] = *(const uint16_t*)p;
    else if constexpr (NB == 4) w[0] = *(const uint32_t*)p;
    else if constexpr (NB == 8) {
        uint2 v = *(const uint2*)p;
        w[0] = v.x;
        w[1] = v.y;
    } else if constexpr (NB == 16) {
        uint4 v = *(const uint4*)p;
        w[0] = v.x;
        w[1] = v.y;
        w[2] = v.z;
        w[3] = v.w;
    } else {
        uint4 v = *(const uint4*)p, u = *(const uint4*)(p + 16);
        w[0] = v.x;
        w[1] = v.y;
        w[2] = v.z;
        w[3] = v.w;
        w[4] = u.x;
        w[5] = u.y;
        w[6] = u.z;
        w[7] = u.w;
    }
}

template <int G>
__device__ inline void storeG(uint8_t* p, uint32_t v0, uint32_t v1)
{
    if constexpr (G == 1) p[0] = uint8_t(v0);
    else if constexpr (G == 2) *(uint16_t*)p = uint16_t(v0);
    else if constexpr (G == 4) *(uint32_t*)p = v0;
    else *(uint2*)p = make_uint2(v0, v1);
}

struct PackLds {
    uint32_t rcode[4][256];     // reversed code | length << 16
    uint64_t pay[4];            // absolute payload offset of each stream
    uint32_t mode[4];
    uint32_t red[kWaves];
    uint32_t tot[4];
};

// Sub-stream passes for one chunk; B, G compile-time.
template <int B, int G>
__device__ void pack_chunk(const uint8_t* __restrict__ src, const uint8_t* __restrict__ base, uint8_t* __restrict__ dst,
                           uint32_t m, uint32_t W, PackLds& P, uint32_t* offs /* [B][W] in LDS */)
{
    int mode[B];
    uint64_t pay_abs[B];
#pragma unroll
    for (int k = 0; k < B; k++) {
        mode[k] = __builtin_amdgcn_readfirstlane(P.mode[k]);
        pay_abs[k] = P.pay[k];
    }
    constexpr int NB = B * G;
    constexpr int NW = NB >= 4 ? NB / 4 : 1;
    const int t = threadIdx.x;
    const uint32_t Gfull = m / G;
    const uint32_t rem = m - Gfull * G;
    const uint32_t Gall = Gfull + (rem ? 1 : 0);
    bool any_huf = false;
#pragma unroll
    for (int k = 0; k < B; k++) any_huf |= mode[k] == kModeHuf;

    // stream byte i of group word array
    auto sym_of = [&](const uint32_t* wd, int k, int i) -> uint32_t {
        const int j = i * B + (B - 1 - k);
        return (wd[j >> 2] >> (8 * (j & 3))) & 0xFFu;
    };
    auto load_words = [&](uint32_t q, uint32_t* wd) {
        const uint32_t e = q * G;
        if (q < Gfull) {
            loadNB<NB>(src + uint64_t(e) * B, wd);
            if (base) {
                uint32_t bw[NW];
                loadNB<NB>(base + uint64_t(e) * B, bw);
#pragma unroll
                for (int x = 0; x < NW; x++) wd[x] ^= bw[x];
            }
        } else {
#pragma unroll
            for (int x = 0; x < NW; x++) wd[x] = 0;
            for (uint32_t j = 0; j < rem * B; j++) {
                uint32_t v = src[uint64_t(e) * B + j] ^ (base ? base[uint64_t(e) * B + j] : 0);
                wd[j >> 2] |= v << (8 * (j & 3));
            }
        }
    };
    const uint32_t head = huf_head(W);
    if (any_huf) {
        // pass A: bit length of every sub-stream
        for (uint32_t w = t; w < W; w += kBlock) {
            uint32_t acc[B];
#pragma unroll
            for (int k = 0; k < B; k++) acc[k] = 0;
            for (uint32_t q = w; q < Gall; q += W) {
                uint32_t wd[NW];
                load_words(q, wd);
                const int cnt = q < Gfull ? G : int(rem);
#pragma unroll
                for (int k = 0; k < B; k++) {
                    if (mode[k] != kModeHuf) continue;
#pragma unroll
                    for (int i = 0; i < G; i++)
                        if (i < cnt) acc[k] += P.rcode[k][sym_of(wd, k, i)] >> 16;
                }
            }
#pragma unroll
            for (int k = 0; k < B; k++) offs[k * W + w] = acc[k];
        }
        __syncthreads();
    }
    // per HUF stream: write the lengths, turn them into start bits in place
    // (block scan), zero the dwords shared by two sub-streams and the padding
#pragma unroll
    for (int k = 0; k < B; k++) {
        if (mode[k] != kModeHuf) continue;
        uint8_t* pay = dst + pay_abs[k];
        uint32_t* bs = (uint32_t*)(pay + head);
        // block-wide exclusive scan over W in chunks of 256
        uint32_t carry = 0;
        for (uint32_t b0 = 0; b0 < W; b0 += kBlock) {
            const uint32_t w = b0 + t;
            const uint32_t l = w < W ? offs[k * W + w] : 0;
            uint32_t inc = l;
            const int lane = t & 63, wv = t >> 6;
#pragma unroll
            for (int dd = 1; dd < 64; dd <<= 1) {
                uint32_t o = __shfl_up(inc, dd, 64);
                if (lane >= dd) inc += o;
            }
            if (lane == 63) P.red[wv] = inc;
            __syncthreads();
            uint32_t pre = carry, tot = carry;
            for (int i = 0; i < kWaves; i++) {
                pre += i < wv ? P.red[i] : 0;
                tot += P.red[i];
            }
            __syncthreads();
            const uint32_t off = pre + inc - l;
            if (w < W) {
                offs[k * W + w] = off;
                ((uint16_t*)(pay + 128))[w] = uint16_t(l);
                bs[off >> 5] = 0;   // dword holding the start of this sub-stream
            }
            carry = tot;
        }
        if (t == 0) P.tot[k] = carry;
        // nibble table
        if (t < 128) pay[t] = uint8_t((P.rcode[k][2 * t] >> 16) | ((P.rcode[k][2 * t + 1] >> 16) << 4));
        // zero pad between the lengths and the bitstream
        for (uint32_t i = 128 + 2 * W + t; i < head; i += kBlock) pay[i] = 0;
        __syncthreads();
        // zero from the dword holding the last bit to the aligned end
        const uint32_t T = P.tot[k];
        const uint32_t end_bytes = uint32_t(align16(head + (T + 7) / 8));
        const uint32_t first_dw = T ? (T - 1) >> 5 : 0;
        for (uint32_t i = first_dw + t; i < (end_bytes - head) / 4; i += kBlock) bs[i] = 0;
    }
    // RAW padding
#pragma unroll
    for (int k = 0; k < B; k++) {
        if (mode[k] != kModeRaw) continue;
        uint8_t* pay = dst + pay_abs[k];
        for (uint32_t i = m + t; i < uint32_t(align16(m)); i += kBlock) pay[i] = 0;
    }
    __threadfence();
    __syncthreads();
    // pass B: codes and raw bytes
    for (uint32_t w = t; w < W; w += kBlock) {
        uint64_t acc[B];
        uint32_t nacc[B], di[B];
        bool first[B];
#pragma unroll
        for (int k = 0; k < B; k++) {
            uint32_t o = (mode[k] == kModeHuf) ? offs[k * W + w] : 0;
            acc[k] = 0;
            nacc[k] = o & 31;
            di[k] = o >> 5;
            first[k] = (o & 31) != 0;
        }
        for (uint32_t q = w; q < Gall; q += W) {
            uint32_t wd[NW];
            load_words(q, wd);
            const int cnt = q < Gfull ? G : int(rem);
            const uint32_t e = q * G;
#pragma unroll
            for (int k = 0; k < B; k++) {
                if (mode[k] == kModeRaw) {
                    uint8_t* pay = dst + pay_abs[k];
                    if (cnt == G) {
                        uint32_t v0 = 0, v1 = 0;
#pragma unroll
                        for (int i = 0; i < G; i++) {
                            if (i < 4) v0 |= sym_of(wd, k, i) << (8 * i);
                            else v1 |= sym_of(wd, k, i) << (8 * (i - 4));
                        }
                        storeG<G>(pay + e, v0, v1);
                    } else {
                        for (int i = 0; i < cnt; i++) pay[e + i] = uint8_t(sym_of(wd, k, i));
                    }
                } else if (mode[k] == kModeHuf) {
                    uint32_t* bs = (uint32_t*)(dst + pay_abs[k] + head);
#pragma unroll
                    for (int i = 0; i < G; i++) {
                        if (i < cnt) {
                            const uint32_t cw = P.rcode[k][sym_of(wd, k, i)];
                            acc[k] |= uint64_t(cw & 0xFFFFu) << nacc[k];
                            nacc[k] += cw >> 16;
                            if (nacc[k] >= 32) {
                                if (first[k]) atomicOr(&bs[di[k]], uint32_t(acc[k]));
                                else bs[di[k]] = uint32_t(acc[k]);
                                first[k] = false;
                                acc[k] >>= 32;
                                nacc[k] -= 32;
                                di[k]++;
                            }
                        }
                    }
                }
            }
        }
#pragma unroll
        for (int k = 0; k < B; k++) {
            if (mode[k] == kModeHuf && nacc[k] > 0) {
                uint32_t* bs = (uint32_t*)(dst + pay_abs[k] + head);
                atomicOr(&bs[di[k]], uint32_t(acc[k]));
            }
        }
    }
}

__global__ __launch_bounds__(kBlock) void k_pack(EncDesc one, const EncDesc* __restrict__ descs, int n_desc,
                                                 const uint32_t* __restrict__ chunk_prefix, uint32_t total_chunks,
                                                 EncParams p, const EncEntry* __restrict__ entries,
                                                 const CodeWord* __restrict__ codes,
                                                 const uint64_t* __restrict__ offsets,
                                                 const uint64_t* __restrict__ totals)
{
    __shared__ PackLds P;
    extern __shared__ uint32_t offs_dyn[];
    const int t = threadIdx.x;
    const uint32_t B = p.B;
    for (uint32_t gc = blockIdx.x; gc < total_chunks; gc += gridDim.x) {
        const int di = descs ? find_desc(chunk_prefix, n_desc, gc) : 0;
        const EncDesc d = descs ? descs[di] : one;
        if (totals[di] > d.dst_cap) continue;   // too small: the host reports it
        const uint32_t c = gc - (descs ? chunk_prefix[di] : 0);
        const uint32_t E = p.chunk / B;
        const uint64_t e0 = uint64_t(c) * E;
        const uint32_t m = uint32_t(min(uint64_t(E), d.n - e0));
        const uint32_t W = (m + p.S - 1) / p.S;
        const uint64_t payload_base = 64 + 16ull * d.n_chunks * B;
        for (uint32_t k = 0; k < B; k++) {
            const uint64_t ei = uint64_t(gc) * B + k;
            const uint32_t mode = entries[ei].mode;
            if (t == 0) {
                P.mode[k] = mode;
                P.pay[k] = payload_base + offsets[ei];
            }
            if (mode == kModeHuf) {
                const uint32_t cw = codes[ei * 256 + t];
                const uint32_t l = cw >> 16;
                P.rcode[k][t] = l ? ((__brev(cw & 0xFFFFu) >> (32 - l)) | (l << 16)) : 0u;
            }
        }
        __syncthreads();
        const uint8_t* src = d.src + e0 * B;
        const uint8_t* base = d.base ? d.base + e0 * B : nullptr;
        switch (B * 16 + p.g) {
#define ZIPNN_CASE(BB, GG)                                                                                 \
    case BB * 16 + GG:                                                                                    \
        pack_chunk<BB, GG>(src, base, d.dst, m, W, P, offs_dyn);                                          \
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
            break;
        }
        __syncthreads();
    }
}

}  // namespace

hipError_t launch_analyze(const EncDesc& one, const EncDesc* d_descs, int n_desc, const uint32_t* d_chunk_prefix,
                          uint32_t total_chunks, const EncParams& p, EncEntry* entries, CodeWord* codes,
                          hipStream_t s)
{
    if (!total_chunks) return hipSuccess;
    const uint32_t grid = min(total_chunks, 1u << 16);
    k_analyze<<<grid, kBlock, 0, s>>>(one, d_descs, n_desc, d_chunk_prefix, total_chunks, p, entries, codes);
    return hipGetLastError();
}

hipError_t launch_place(const EncDesc& one, const EncDesc* d_descs, int n_desc, const EncParams& p,
                        const EncEntry* entries, uint64_t* d_offsets, uint64_t* d_totals, hipStream_t s)
{
    k_place<<<n_desc, kBlock, 0, s>>>(one, d_descs, p, entries, d_offsets, d_totals);
    return hipGetLastError();
}

hipError_t launch_pack(const EncDesc& one, const EncDesc* d_descs, int n_desc, const uint32_t* d_chunk_prefix,
                       uint32_t total_chunks, const EncParams& p, const EncEntry* entries, const CodeWord* codes,
                       const uint64_t* offsets, const uint64_t* d_totals, hipStream_t s)
{
    if (!total_chunks) return hipSuccess;
    const uint32_t grid = min(total_chunks, 1u << 16);
    const uint32_t Wmax = (p.chunk / p.B + p.S - 1) / p.S;
    const size_t lds = size_t(p.B) * Wmax * sizeof(uint32_t);
    k_pack<<<grid, kBlock, lds, s>>>(one, d_descs, n_desc, d_chunk_prefix, total_chunks, p, entries, codes, offsets,
                                     d_totals);
    return hipGetLastError();
}

}  // namespace zipnn
