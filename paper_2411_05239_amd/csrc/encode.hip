// Encode kernels of the gfx950 ZipNN codec.
//
//   k_analyze  one workgroup per chunk: reads the chunk (16-byte loads, XOR
//              with the base for a delta, paper §IV-B, exponent extraction
//              when asked, §III-A), splits every word into its B byte groups
//              (paper §III-A/§III-B) and histograms each group in LDS; wave k
//              then builds the code of group k: optimal lengths <= L by
//              package-merge (Larmore & Hirschberg, computed with parallel
//              ranks, see build_lengths) and canonical codes (RFC 1951
//              §3.2.2).  A group with one value becomes RLE (paper §III-B);
//              a group whose most frequent byte fills half of it is also a ZG
//              candidate (zero-aware coding, §IV-B).  For every candidate the
//              four waves sum each lane's code bits lane group by lane
//              group, which gives the exact payload sizes, so
//              AUTO keeps the smallest of RAW, HUF and ZG (paper §III-B, §V-A).
//              With a probe interval the probe chunks run first
//              (compressibility probing, §III-B).
//   k_place    one workgroup per tensor: exclusive scan of the 128-byte aligned
//              payload sizes in chunk-major order -> map entries and header
//              (the map that enables parallel decode, paper §V-A), and whether
//              the map holds ZG entries (a header flag).
//   k_pack     one workgroup per chunk: raw groups are copied with 16-byte
//              stores; for a Huffman or ZG group, wave v writes lane groups v,
//              v+4, ...: its lanes replay the same steps, and in every round
//              the lanes that the decoder will serve write their next word to
//              consecutive slots (ballot + prefix popcount), encoding codes
//              ahead of the decoder model.  Every byte of the payload extent,
//              padding included, is written; no atomics.
#include <type_traits>

#include "zipnn_internal.h"

namespace zipnn {
namespace {

constexpr int kWaves = kBlock / 64;
// The counting pass's histograms: kRep copies for all byte groups together
// (16 / B copies of each), shared by the workgroup's waves; lane l of every
// wave adds to copy l / (64 B / 16) of its group, whose bins start kRepShift *
// copy words further on.  Lanes holding one value hit at most 4 B of the
// same address in an instruction instead of 64 (LDS atomics on one address
// serialise), and the shift puts the copies' equal bins on different banks.
constexpr int kRep = 16;
constexpr int kRepStride = 288;   // 256 bins + room for the shift

struct PmWave {                 // package-merge workspace of one wave
    alignas(16) uint32_t leafw[256];   // leaf weights, ascending (f, symbol)
    uint16_t leafsym[256];
    alignas(16) uint32_t pk[256];      // package weights of the current level
    union {
        alignas(16) uint32_t key[256];   // the sort keys, used before the lists
        uint32_t cur[512];               // current list weights
    };
    uint32_t leafbits[kMaxL][16];   // bit p: item p of the list of a level is a leaf
    uint8_t len[256];           // code length per symbol
};

// Sized by the word width B (wave k < B builds the code of byte group k), so
// that a BF16 workgroup takes 22 KB and seven fit on a CU.
template <int B>
union AnalyzeLds {
    uint32_t rep[kRep][kRepStride];  // the counting pass's histogram copies
    uint32_t hist[kWaves][B][256];   // per-wave sub-histograms (the ZG counting pass)
    PmWave pm[B];                    // per-group code construction
    uint32_t lgw[2][4][64];          // words per lane group: HUF, ZG (replay)
};

__device__ inline uint32_t wave_sum(uint32_t v)
{
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d, 64);
    return v;
}

// number of items of a sorted u32 array a[0..n) that are < x (strict) or <= x.
// Up to 64 items (n uniform): a scan of 16-byte LDS reads, four in flight
// (every lane of the wave reads the same words: a broadcast), instead of a
// chain of dependent reads; a[] must be 16-byte aligned and hold 64 items.
template <bool LE>
__device__ inline uint32_t count_small(const uint32_t* a, uint32_t n, uint32_t x)
{
    const uint4* v = reinterpret_cast<const uint4*>(a);
    uint32_t c = 0;
#pragma unroll 4
    for (uint32_t q = 0; q < 16; q++) {
        const uint4 y = v[q];
        const uint32_t i = 4 * q;
        c += uint32_t(i < n && (LE ? y.x <= x : y.x < x)) + uint32_t(i + 1 < n && (LE ? y.y <= x : y.y < x)) +
             uint32_t(i + 2 < n && (LE ? y.z <= x : y.z < x)) + uint32_t(i + 3 < n && (LE ? y.w <= x : y.w < x));
    }
    return c;
}
__device__ inline uint32_t count_lt(const uint32_t* a, uint32_t n, uint32_t x)
{
    if (n <= 64) return count_small<false>(a, n, x);
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
    if (n <= 64) return count_small<true>(a, n, x);
    uint32_t lo = 0, hi = n;
    while (lo < hi) {
        uint32_t mid = (lo + hi) >> 1;
        if (a[mid] <= x) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

// Optimal code lengths <= L for the histogram held in registers (fv[r] =
// f[lane + 64 r], at least two symbols with f > 0, `tot` = sum of f) into
// P.len, by one wave.  With `shortcut` (policy AUTO) it returns false as soon
// as a lower bound of the payload (`head` bytes + the coded bits) shows that
// it cannot be smaller than `raw` bytes; the lengths are then not built.
//
// Package-merge with lists made of leaves and packages: list 0 = the leaves
// sorted by (f, symbol); list d = the leaves merged with the packages of
// consecutive pairs of list d-1, a leaf before a package of equal weight.
// Merging two sorted sequences is done by ranks: leaf i lands at
// i + #{packages lighter than it}, package j at j + #{leaves not heavier}.
// The 2n'-2 first items of the top list are selected; the packages among the
// first m items of a list select the first 2*(their count) items of the list
// below; leaf i is selected at a level iff i < (leaves among the selected
// items), so its length is the number of such levels.  Each level keeps a
// 512-bit mask of the list positions that hold leaves, so that count is a
// popcount (16 words per level instead of a position per leaf: the LDS of a
// workgroup fits four per CU).
__device__ __attribute__((always_inline)) bool build_lengths(const uint32_t* fv, uint32_t tot, uint32_t raw, uint32_t head, uint32_t L,
                              bool shortcut, PmWave& P, uint32_t& T_out)
{
    T_out = 0;
    const int lane = threadIdx.x & 63;
    uint32_t d = 0;
#pragma unroll
    for (int r = 0; r < 4; r++) d += __popcll(__ballot(fv[r] > 0));
    if (shortcut) {
        // Any prefix code spends at least the empirical entropy, sum f log2(tot/f)
        // bits.  If even that bound gives a payload no smaller than the raw
        // bytes, AUTO cannot keep this code (the decision is the one the exact
        // size would give), and it need not be built.  In single precision
        // (v_log_f32): each log2 of a count below 2^23 is within about 2^-18
        // of the truth, so the terms err by under 10^-5 bits per symbol in
        // all, and rounding the products and the sum errs by under 10^-6 of
        // the sum; the margins below (10^-4 relative, 10^-4 bits per symbol)
        // keep the bound a lower bound.  Near the boundary the code is built
        // and sized exactly, as without the test.
        const float lt = __log2f(float(tot));
        float h = 0.0f;
#pragma unroll
        for (int r = 0; r < 4; r++)
            if (fv[r]) h += float(fv[r]) * (lt - __log2f(float(fv[r])));
#pragma unroll
        for (int o = 32; o >= 1; o >>= 1) h += __shfl_xor(h, o, 64);
        const float lb = h * (1.0f - 1e-4f) - 1e-4f * float(tot) - 1.0f;
        const uint64_t words_lb = lb > 0.0f ? uint64_t(lb / 32.0f) : 0u;   // floor: a lower bound too
        if (uint64_t(head) + 4 * words_lb >= raw) return false;
    }
    // sort the leaves by key = f << 8 | symbol (f < 2^24 since m <= 2^22)
#pragma unroll
    for (int r = 0; r < 4; r++) P.key[lane + 64 * r] = fv[r] ? ((fv[r] << 8) | uint32_t(lane + 64 * r)) : 0xFFFFFFFFu;
    __builtin_amdgcn_wave_barrier();
    {
        // rank of each key among all 256 (keys are distinct): four keys per
        // 16-byte LDS read, shared by the lane's four symbols
        uint32_t k4[4], rank[4] = {0, 0, 0, 0};
#pragma unroll
        for (int r = 0; r < 4; r++) k4[r] = P.key[lane + 64 * r];
        const uint4* kv = reinterpret_cast<const uint4*>(P.key);
#pragma unroll 4
        for (int s = 0; s < 64; s++) {
            const uint4 kk = kv[s];
#pragma unroll
            for (int r = 0; r < 4; r++)
                rank[r] += uint32_t(kk.x < k4[r]) + uint32_t(kk.y < k4[r]) + uint32_t(kk.z < k4[r]) +
                           uint32_t(kk.w < k4[r]);
        }
#pragma unroll
        for (int r = 0; r < 4; r++) {
            if (fv[r]) {
                P.leafw[rank[r]] = fv[r];
                P.leafsym[rank[r]] = uint16_t(lane + 64 * r);
            }
        }
    }
    __builtin_amdgcn_wave_barrier();
    const uint32_t n = d;
    // level 0: the leaves alone
    for (uint32_t i = lane; i < n; i += 64) P.cur[i] = P.leafw[i];
    for (uint32_t x = lane; x < kMaxL * 16; x += 64) {
        const uint32_t lo = 32 * (x & 15);
        (&P.leafbits[0][0])[x] = x < 16 ? (n >= lo + 32 ? ~0u : (n > lo ? (1u << (n - lo)) - 1u : 0u)) : 0u;
    }
    uint32_t curlen = n;
    __builtin_amdgcn_wave_barrier();
    for (uint32_t lev = 1; lev < L; lev++) {
        const uint32_t npk = curlen / 2;
        for (uint32_t j = lane; j < npk; j += 64) P.pk[j] = P.cur[2 * j] + P.cur[2 * j + 1];
        __builtin_amdgcn_wave_barrier();
        for (uint32_t i = lane; i < n; i += 64) {
            uint32_t p = i + count_lt(P.pk, npk, P.leafw[i]);
            atomicOr(&P.leafbits[lev][p >> 5], 1u << (p & 31));
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
        // leaves among the first sel items of the level's list
        uint32_t c = 0;
        if (lane < 16) {
            const uint32_t lo = 32u * uint32_t(lane), wbits = P.leafbits[lev][lane];
            c = sel >= lo + 32 ? __popc(wbits) : (sel > lo ? __popc(wbits & ((1u << (sel - lo)) - 1u)) : 0u);
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
    T_out = T;
    __builtin_amdgcn_wave_barrier();
    // the payload holds at least its head and ceil(T/8) bytes
    return !(shortcut && head + (T + 7) / 8 >= raw);
}

// Canonical codes (RFC 1951 §3.2.2) of the lengths len[256], by one wave:
// codes[s] = code | length << 16 (0 for absent symbols).  The first code of
// each length follows from the counts of the shorter ones; within a length
// the codes follow the symbol order.
__device__ __attribute__((always_inline)) void canonical_codes(const uint8_t* len, uint32_t L, CodeWord* codes)
{
    const int lane = threadIdx.x & 63;
    uint32_t l4[4];
#pragma unroll
    for (int r = 0; r < 4; r++) l4[r] = len[lane + 64 * r];
    const uint64_t lt_mask = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    uint32_t code4[4] = {0, 0, 0, 0};
    uint32_t first = 0, prev = 0;
    for (uint32_t l = 1; l <= L; l++) {
        first = (first + prev) << 1;
        uint32_t run = 0;
#pragma unroll
        for (int r = 0; r < 4; r++) {
            const uint64_t msk = __ballot(l4[r] == l);
            if (l4[r] == l) code4[r] = first + run + __popcll(msk & lt_mask);
            run += __popcll(msk);
        }
        prev = run;
    }
#pragma unroll
    for (int r = 0; r < 4; r++) codes[lane + 64 * r] = l4[r] ? (code4[r] | (l4[r] << 16)) : 0u;
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

// Load NB bytes (NB in {2,4,8,16,32,64}) from p into 32-bit words.
template <int NB>
__device__ inline void loadNB(const uint8_t* p, uint32_t* w)
{
    if constexpr (NB == 2) w[0] = *(const uint16_t*)p;
    else if constexpr (NB == 4) w[0] = *(const uint32_t*)p;
    else if constexpr (NB == 8) {
        uint2 v = *(const uint2*)p;
        w[0] = v.x;
        w[1] = v.y;
    } else {
#pragma unroll
        for (int i = 0; i < NB / 16; i++) {
            uint4 v = *(const uint4*)(p + 16 * i);
            w[4 * i] = v.x;
            w[4 * i + 1] = v.y;
            w[4 * i + 2] = v.z;
            w[4 * i + 3] = v.w;
        }
    }
}

// The words of group q of a chunk (g elements, XORed with the base, then with
// the exponent extracted when xf), or of the partial last group (zero beyond
// the chunk's m elements).
template <int B, int G>
__device__ inline void group_words(const uint8_t* src, const uint8_t* base, uint32_t q, uint32_t m, uint32_t* wd,
                                   bool xf)
{
    constexpr int NB = B * G;
    constexpr int NW = NB >= 4 ? NB / 4 : 1;
    const uint32_t e = q * G;
    if (e + G <= m) {
        loadNB<NB>(src + uint64_t(e) * B, wd);
        if (base) {
            uint32_t bw[NW];
            loadNB<NB>(base + uint64_t(e) * B, bw);
#pragma unroll
            for (int x = 0; x < NW; x++) wd[x] ^= bw[x];
        }
    } else {
        // the partial last group: bytes past the chunk's m elements are zero
        const uint32_t nb = (m - e) * B;
#pragma unroll
        for (int x = 0; x < NW; x++) {
            wd[x] = 0;
#pragma unroll
            for (int b = 0; b < 4; b++) {
                const uint32_t jb = 4 * x + b;
                if (jb < nb) {
                    const uint32_t v = src[uint64_t(e) * B + jb] ^ (base ? base[uint64_t(e) * B + jb] : 0u);
                    wd[x] |= v << (8 * b);
                }
            }
        }
    }
    if (xf)
#pragma unroll
        for (int x = 0; x < NW; x++) wd[x] = exp_fwd<B>(wd[x]);
}

// Element e of a chunk as a little-endian word (XORed with the base, exponent
// extracted when xf), read byte by byte.
template <int B>
__device__ inline uint32_t element_word(const uint8_t* src, const uint8_t* base, uint32_t e, bool xf)
{
    uint32_t v = 0;
#pragma unroll
    for (int b = 0; b < B; b++) {
        const uint64_t o = uint64_t(e) * B + b;
        v |= uint32_t(src[o] ^ (base ? base[o] : 0u)) << (8 * b);
    }
    return xf ? exp_fwd<B>(v) : v;
}

// byte of stream k of element i of a group's words
template <int B>
__device__ inline uint32_t sym_of(const uint32_t* wd, int k, int i)
{
    const int jb = i * B + (B - 1 - k);
    return (wd[jb >> 2] >> (8 * (jb & 3))) & 0xFFu;
}

// Whether a group of gcnt symbols of stream k holds a value other than z.
template <int B, int G>
__device__ inline bool marked(const uint32_t* wd, int k, uint32_t gcnt, uint32_t z)
{
    bool mk = false;
#pragma unroll
    for (int i = 0; i < G; i++) mk |= uint32_t(i) < gcnt && sym_of<B>(wd, k, i) != z;
    return mk;
}

// Histograms of the ZG candidates (bit k of zc, fill value z[k]) over the
// groups that hold a value other than z: h[k][s] of this wave, except the
// count of z itself, which is returned per stream (summed over the wave).
template <int B, int G>
__device__ __attribute__((always_inline)) void zg_count(const uint8_t* src, const uint8_t* base, uint32_t zc, const uint32_t* z, uint32_t m,
                         uint32_t (*h)[256], uint32_t* zcount, bool xf)
{
    constexpr int NB = B * G;
    constexpr int NW = NB >= 4 ? NB / 4 : 1;
    constexpr uint32_t CB = 4;   // groups in flight per thread
    const uint32_t Gtot = (m + G - 1) / G;
    uint32_t nz[B];
#pragma unroll
    for (int k = 0; k < B; k++) nz[k] = 0;
    for (uint32_t q0 = threadIdx.x; q0 < Gtot; q0 += CB * kBlock) {
        uint32_t wds[CB][NW];
#pragma unroll
        for (uint32_t u = 0; u < CB; u++)
            if (q0 + u * kBlock < Gtot) group_words<B, G>(src, base, q0 + u * kBlock, m, wds[u], xf);
#pragma unroll
        for (uint32_t u = 0; u < CB; u++) {
            const uint32_t q = q0 + u * kBlock;
            if (q >= Gtot) continue;
            const uint32_t gcnt = min(uint32_t(G), m - q * G);
#pragma unroll
            for (int k = 0; k < B; k++) {
                if (!((zc >> k) & 1) || !marked<B, G>(wds[u], k, gcnt, z[k])) continue;
#pragma unroll
                for (int i = 0; i < G; i++) {
                    if (uint32_t(i) >= gcnt) continue;
                    const uint32_t v = sym_of<B>(wds[u], k, i);
                    if (v == z[k]) nz[k]++;
                    else atomicAdd(&h[k][v], 1u);
                }
            }
        }
    }
#pragma unroll
    for (int k = 0; k < B; k++) zcount[k] = wave_sum(nz[k]);
}

// Bytes of stream k of the g elements of a group's words, packed little-endian
// into one register (groups of at most 4 bytes per stream): v_perm_b32 picks
// byte B-1-k of each word (selector 0-3: the second operand, 4-7: the first,
// 0x0C: zero).
template <int B, int G>
__device__ inline uint32_t gather_stream(const uint32_t* wd, int k)
{
    if constexpr (B == 2) {
        const uint32_t b = uint32_t(1 - k);   // byte of the 16-bit element
        if constexpr (G == 2) return __builtin_amdgcn_perm(0u, wd[0], 0x0C0C0000u | ((b + 2) << 8) | b);
        else return __builtin_amdgcn_perm(wd[1], wd[0], ((b + 6) << 24) | ((b + 4) << 16) | ((b + 2) << 8) | b);
    } else if constexpr (B == 4) {
        const uint32_t b = uint32_t(3 - k);
        const uint32_t lo = __builtin_amdgcn_perm(wd[1], wd[0], 0x0C0C0000u | ((b + 4) << 8) | b);
        if constexpr (G == 2) return lo;
        else return lo | __builtin_amdgcn_perm(wd[3], wd[2], ((b + 4) << 24) | (b << 16) | 0x0C0Cu);
    } else {
        uint32_t v = 0;
#pragma unroll
        for (int i = 0; i < G; i++) v |= sym_of<B>(wd, k, i) << (8 * i);
        return v;
    }
}

// Count the words each candidate's lane group j of one chunk takes: HUF
// candidates (bit k of hc, lengths lens[k]) over every group, ZG candidates
// (bit k of zgc, lengths lens2[k], fill value z[k]) over the groups holding
// another value.  A lane's count follows from its code bits and those of its
// last pair alone (see the end of the function).  Lane 0 of the wave writes
// the counts to lgw[0][k][j] and lgw[1][k][j].
template <int B, int G>
__device__ __attribute__((always_inline)) void count_lane_group(const uint8_t* src, const uint8_t* base, uint32_t hc, uint32_t zgc,
                                 const uint8_t (*lens)[256], const uint8_t (*lens2)[256], const uint32_t* z,
                                 uint32_t L, uint32_t j, uint32_t W, uint32_t m, uint32_t (*lgw)[4][64], bool xf)
{
    constexpr int NB = B * G;
    constexpr int NW = NB >= 4 ? NB / 4 : 1;
    const uint32_t lane = threadIdx.x & 63;
    const uint32_t w = 64 * j + lane;
    const uint32_t Gtot = (m + G - 1) / G, Gfull = m / G, rem = m - Gfull * G;
    const uint32_t ng = (w < W && w < Gtot) ? (Gtot - 1 - w) / W + 1 : 0;
    // per candidate: the lane's code bits and those of its last pair (a lane
    // with no pair takes no word)
    uint32_t bits[2][B], last[2][B];
#pragma unroll
    for (int k = 0; k < B; k++) bits[0][k] = bits[1][k] = last[0][k] = last[1][k] = 0;
    constexpr uint32_t CB = 4;   // groups in flight per lane
    for (uint32_t j0 = 0; j0 < ng; j0 += CB) {
        uint32_t wds[CB][NW];
#pragma unroll
        for (uint32_t u = 0; u < CB; u++)
            if (j0 + u < ng) group_words<B, G>(src, base, w + (j0 + u) * W, m, wds[u], xf);
#pragma unroll
        for (uint32_t u = 0; u < CB; u++) {
            const uint32_t jj = j0 + u;
            const uint32_t q = w + jj * W;
            const uint32_t gcnt = jj >= ng ? 0u : (q < Gfull ? G : rem);
            const uint32_t* wd = wds[u];
#pragma unroll
            for (int k = 0; k < B; k++) {
#pragma unroll
                for (int v = 0; v < 2; v++) {
                    if (!(((v ? zgc : hc) >> k) & 1)) continue;
                    const uint8_t* ln = v ? lens2[k] : lens[k];
                    const uint32_t gc = (v && !marked<B, G>(wd, k, gcnt, z[k])) ? 0u : gcnt;
#pragma unroll
                    for (int pr = 0; pr < G / 2; pr++) {
                        if (2u * pr < gc) {
                            uint32_t c = ln[sym_of<B>(wd, k, 2 * pr)];
                            if (2u * pr + 1 < gc) c += ln[sym_of<B>(wd, k, 2 * pr + 1)];
                            bits[v][k] += c;
                            last[v][k] = c;
                        }
                    }
                }
            }
        }
    }
    // before each pair a lane holding fewer than 2L bits takes a word, so
    // after that check 32 * taken - consumed lies in [2L, 2L + 31]: a lane
    // takes ceil((consumed before its last pair + 2L) / 32) words in all
#pragma unroll
    for (int k = 0; k < B; k++) {
#pragma unroll
        for (int v = 0; v < 2; v++) {
            const uint32_t req = bits[v][k] ? (bits[v][k] - last[v][k] + 2 * L + 31) / 32 : 0u;
            const uint32_t tot = wave_sum(req);
            if (lane == 0) lgw[v][k][j] = tot;
        }
    }
}

template <int B>
struct AnalyzeTail {
    uint8_t lens[B][256];    // HUF code lengths
    uint8_t lens2[B][256];   // ZG code lengths
    uint32_t z[4];           // ZG fill value: the most frequent byte (smallest on ties)
    uint32_t open;           // bit k: mode still to be decided (neither forced RAW nor RLE)
    uint32_t hc;             // bit k: HUF candidate
    uint32_t zc;             // bit k: ZG considered (histogram over marked groups needed)
    uint32_t zgc;            // bit k: ZG candidate
    uint32_t fin;            // bit k: ZG chosen (else HUF) for a coded stream
    uint32_t coded;          // bit k: coded (HUF or ZG chosen)
    uint32_t words[2][4];    // words over all lane groups, per stream: HUF, ZG
    uint32_t T[2][4];        // coded bits of the candidates: HUF, ZG
    int pol[4];              // policy of each group in this chunk (RAW where probing skips it)
    uint32_t specok;         // bit k: the main pass's count of zeros in marked groups holds (z = 0)
    uint32_t amb;            // staged packing: bit k, the mode decision needs exact sizes
};

// One workgroup per chunk (phase -1: every chunk; with a probe interval K,
// phase 0: the probe chunks c mod (K+1) = 0 of each tensor, phase 1: the
// others, where a byte group that the run's probe chunk stored raw is stored
// raw without analysis under AUTO: compressibility probing, paper §III-B):
//   1. histogram f of every byte group;
//   2. wave k classifies group k: forced RAW, RLE (one value), else HUF
//      lengths of f (unless ZG is forced) and, when ZG is forced or (AUTO)
//      the most frequent value z fills half the group, a ZG candidate;
//   3. for ZG candidates: histogram over the groups of g symbols that hold a
//      value other than z, and ZG lengths of it;
//   4. the four waves count the words of every candidate lane group by lane
//      group for every candidate, which gives the exact sizes;
//   5. the mode of each group (AUTO: the smallest of RAW, HUF, ZG, ties to
//      RAW then HUF), its entry, its lane-group word counts and its canonical
//      code table.
// (analyze_chunk below; k_analyze runs it over the chunks, k_analyze_pack
// packs each chunk after it.)

// Shared memory of the analysis of one chunk.
template <int BB>
struct AnalyzeShared {
    AnalyzeLds<BB> S;
    uint32_t hist[BB][256];
    AnalyzeTail<BB> A;
    uint32_t zsum[kWaves][4];
    uint32_t zspec[kWaves][4];
};

// The analysis of chunk gc by one workgroup (steps 1-5 above).  Returns
// false when the probing phase leaves the chunk to the other launch.
template <int BB>
__device__ __attribute__((always_inline)) bool analyze_chunk(uint32_t gc, const EncDesc* __restrict__ descs,
                                                             int n_desc, const uint32_t* __restrict__ chunk_prefix,
                                                             const EncParams& p, int phase,
                                                             EncEntry* __restrict__ entries, CodeWord* __restrict__ codes,
                                                             uint32_t* __restrict__ nwords, AnalyzeShared<BB>& sh)
{
    AnalyzeLds<BB>& S = sh.S;
    auto& hist = sh.hist;
    AnalyzeTail<BB>& A = sh.A;
    auto& zsum = sh.zsum;
    auto& zspec = sh.zspec;
    const int t = threadIdx.x, wv = t >> 6, lane = t & 63;
    constexpr uint32_t B = BB;
    const int di = find_desc(chunk_prefix, n_desc, gc);
    const EncDesc d = descs[di];
    const uint32_t c = gc - chunk_prefix[di];
    const uint32_t run = p.skip + 1;
    const bool probe = c % run == 0;
    if ((phase == 0 && !probe) || (phase == 1 && probe)) return false;
    // the groups this chunk analyses (uniform: every thread reads the same entries)
    uint32_t live = (1u << B) - 1;
    if (!probe)
        for (uint32_t k = 0; k < B; k++)
            if (p.policy[k] == ZIPNN_AUTO && entries[uint64_t(gc - c % run) * B + k].mode == kModeRaw)
                live &= ~(1u << k);
    const uint32_t E = p.chunk / B;
    const uint64_t e0 = uint64_t(c) * E;
    const uint32_t m = uint32_t(min(uint64_t(E), d.n - e0));
    const uint32_t W = (m + p.S - 1) / p.S;
    const uint32_t NG = (W + 63) / 64;
    const uint32_t head = huf_head(W), head_z = head + zg_bitmap(m, p.g);
    if (live == 0) {
        if (uint32_t(t) < B) {
            EncEntry e;
            e.pad = 0;
            e.mode = kModeRaw;
            e.rle = 0;
            e.bytes = m;
            entries[uint64_t(gc) * B + t] = e;
        }
        return true;
    }
    for (uint32_t i = t; i < kRep * kRepStride; i += kBlock) (&S.rep[0][0])[i] = 0;
    if (t == 0) A.open = A.hc = A.zc = A.zgc = A.fin = A.coded = A.specok = A.amb = 0;
    if (t < 8) (&A.words[0][0])[t] = 0;
    if (t < 4) A.pol[t] = ((live >> t) & 1) ? int(p.policy[t]) : ZIPNN_RAW;
    __syncthreads();
    const uint8_t* src = d.src + e0 * B;
    const uint8_t* base = d.base ? d.base + e0 * B : nullptr;
    const uint32_t nbytes = m * B;
    const bool xf = (p.flags & kFlagExp) != 0;
    // this lane's copy of every byte group's histogram
    constexpr uint32_t R = kRep / B;
    const uint32_t rc = uint32_t(lane) / (64 / R);
    const uint32_t rshift = rc * (32 / R);
    auto bin = [&](uint32_t k, uint32_t v) { return &S.rep[k * R + rc][v + rshift]; };
    // 16-byte vectors; the element boundary is aligned since 16 % B == 0
    const uint32_t nvec = nbytes / 16;
    // a stream whose bytes agree across an eighth of the wave's lanes in
    // the first vector is taken as skewed: there, the lanes holding the
    // first active lane's value add together, since LDS atomics on one
    // bin serialise (the rule only changes how the counts are summed)
    uint32_t skew = 0;
    if (uint32_t(t) < nvec) {
        uint4 x = ((const uint4*)src)[t];
        if (base) {
            const uint4 y = ((const uint4*)base)[t];
            x.x ^= y.x;
        }
        if (xf) x.x = exp_fwd<B>(x.x);
        for (uint32_t k = 0; k < B; k++) {
            const uint32_t byte = (x.x >> (8 * (B - 1 - k))) & 0xFFu;
            const uint32_t hot = __builtin_amdgcn_readfirstlane(byte);
            if (__popcll(__ballot(byte == hot)) >= 8) skew |= 1u << k;
        }
    }
    skew = __builtin_amdgcn_readfirstlane(skew);
    // Delta-like groups (zero bytes in at least half of the first 64
    // vectors; the same vectors in every wave, so the choice is uniform)
    // also count, in this pass, the zero bytes that lie in groups of g
    // holding a nonzero byte.  Every nonzero byte lies in such a group, so
    // if 0 turns out to be the most frequent value, the ZG histogram is
    // this pass's histogram with that count in place of the count of 0,
    // and the ZG pass over the data is not needed.
    uint32_t spec = 0;
    if (nbytes % 16 == 0 && p.g * B <= 16) {
        uint32_t x0 = 0;
        if (uint32_t(lane) < nvec) {
            x0 = ((const uint32_t*)src)[4 * lane];
            if (base) x0 ^= ((const uint32_t*)base)[4 * lane];
            if (xf) x0 = exp_fwd<B>(x0);
        }
        for (uint32_t k = 0; k < B; k++) {
            const uint32_t byte = (x0 >> (8 * (B - 1 - k))) & 0xFFu;
            const bool zg_policy = A.pol[k] == ZIPNN_AUTO || A.pol[k] == ZIPNN_ZG;
            if (zg_policy && __popcll(__ballot(uint32_t(lane) < nvec && byte == 0)) >= 32) spec |= 1u << k;
        }
    }
    spec = __builtin_amdgcn_readfirstlane(spec);
    uint32_t zin[4] = {0, 0, 0, 0};   // zero bytes in marked groups, per group of bytes
    const uint32_t G = p.g;
    // SK: the skewed streams, known here (or -1: tested per byte)
    // LV: every group is live (no per-byte test)
    // SP: count the zeros in marked groups of the streams in `spec`
    auto count = [&](auto sk_const, auto lv_const, auto sp_const) {
        constexpr int SK = decltype(sk_const)::value;
        constexpr bool LV = decltype(lv_const)::value;
        constexpr bool SP = decltype(sp_const)::value;
        constexpr uint32_t HB = 4;   // vectors in flight per lane (with the base: 8 loads)
        for (uint32_t v0 = t; v0 < nvec; v0 += HB * kBlock) {
          uint4 xs[HB];
#pragma unroll
          for (uint32_t i = 0; i < HB; i++) {
              const uint32_t v = v0 + i * kBlock;
              if (v < nvec) {
                  xs[i] = ((const uint4*)src)[v];
                  if (base) {
                      const uint4 y = ((const uint4*)base)[v];
                      xs[i].x ^= y.x;
                      xs[i].y ^= y.y;
                      xs[i].z ^= y.z;
                      xs[i].w ^= y.w;
                  }
                  if (xf) {
                      xs[i].x = exp_fwd<B>(xs[i].x);
                      xs[i].y = exp_fwd<B>(xs[i].y);
                      xs[i].z = exp_fwd<B>(xs[i].z);
                      xs[i].w = exp_fwd<B>(xs[i].w);
                  }
              }
          }
#pragma unroll
          for (uint32_t i = 0; i < HB; i++) {
            if (v0 + i * kBlock < nvec) {
            const uint32_t wds[4] = {xs[i].x, xs[i].y, xs[i].z, xs[i].w};
#pragma unroll
            for (int jb = 0; jb < 16; jb++) {
                const uint32_t byte = (wds[jb >> 2] >> (8 * (jb & 3))) & 0xFF;
                const int k = int(B) - 1 - (jb % int(B));   // byte jb%B of a word -> stream B-1-jb%B
                if (!LV && !((live >> k) & 1)) continue;
                const bool sk = SK >= 0 ? ((SK >> k) & 1) != 0 : ((skew >> k) & 1) != 0;
                if (sk) {
                    const uint32_t hot = __builtin_amdgcn_readfirstlane(byte);
                    const uint64_t msk = __ballot(byte == hot);
                    if (byte != hot) atomicAdd(bin(k, byte), 1u);
                    else if (__builtin_amdgcn_mbcnt_hi(uint32_t(msk >> 32),
                                                       __builtin_amdgcn_mbcnt_lo(uint32_t(msk), 0u)) == 0)
                        atomicAdd(bin(k, hot), uint32_t(__popcll(msk)));
                } else {
                    atomicAdd(bin(k, byte), 1u);
                }
            }
            if constexpr (SP) {
#pragma unroll
                for (int k = 0; k < int(B); k++) {
                    if (!((spec >> k) & 1)) continue;
                    uint32_t nz = 0;   // bit e: element e's byte of group k is nonzero
#pragma unroll
                    for (int e = 0; e < 16 / int(B); e++) {
                        const int jb = e * int(B) + (int(B) - 1 - k);
                        nz |= uint32_t(((wds[jb >> 2] >> (8 * (jb & 3))) & 0xFFu) != 0) << e;
                    }
                    uint32_t mk = 0;   // bit e: element e's group of g holds a nonzero byte
                    for (uint32_t g0 = 0; g0 < 16 / B; g0 += G) {
                        const uint32_t gm = ((1u << G) - 1) << g0;
                        if (nz & gm) mk |= gm;
                    }
                    zin[k] += __popc(mk & ~nz);
                }
            }
            }
          }
        }
    };
    {
        using std::integral_constant;
        using T = integral_constant<bool, true>;
        using F = integral_constant<bool, false>;
        if (live != (1u << B) - 1) count(integral_constant<int, -1>{}, F{}, F{});
        else if (spec) count(integral_constant<int, -1>{}, T{}, T{});
        else if (skew == 0) count(integral_constant<int, 0>{}, T{}, F{});
        else if (skew == 1) count(integral_constant<int, 1>{}, T{}, F{});
        else if (B >= 2 && skew == 3) count(integral_constant<int, B >= 2 ? 3 : -1>{}, T{}, F{});
        else count(integral_constant<int, -1>{}, T{}, F{});
    }
    if (spec)
        for (uint32_t k = 0; k < B; k++) {
            const uint32_t zs = wave_sum(zin[k]);
            if (lane == 0) zspec[wv][k] = zs;
        }
    // the elements after the last whole vector
    for (uint32_t e = nvec * 16 / B + t; e < m; e += kBlock) {
        const uint32_t v = element_word<B>(src, base, e, xf);
        for (uint32_t b = 0; b < B; b++)
            if ((live >> (B - 1 - b)) & 1) atomicAdd(bin(B - 1 - b, (v >> (8 * b)) & 0xFFu), 1u);
    }
    __syncthreads();
    for (uint32_t i = t; i < B * 256; i += kBlock) {
        const uint32_t k = i >> 8, s = i & 255;
        uint32_t v = 0;
        for (uint32_t r = 0; r < R; r++) v += S.rep[k * R + r][s + r * (32 / R)];
        hist[k][s] = v;
    }
    __syncthreads();
    // 2. classification and HUF lengths, wave k for group k
    if (uint32_t(wv) < B) {
        const int k = wv;
        const int policy = A.pol[k];
        uint32_t fv[4], d = 0, best = 0, arg = 0;
#pragma unroll
        for (int r = 0; r < 4; r++) {
            fv[r] = hist[k][lane + 64 * r];
            d += __popcll(__ballot(fv[r] > 0));
            // most frequent value, smallest on ties: key f << 8 | (255 - s)
            const uint32_t key = (fv[r] << 8) | uint32_t(255 - (lane + 64 * r));
            if (key > best) best = key;
        }
#pragma unroll
        for (int o = 32; o >= 1; o >>= 1) best = max(best, uint32_t(__shfl_xor(best, o, 64)));
        arg = 255 - (best & 0xFFu);
        const uint64_t ei = uint64_t(gc) * B + k;
        if (policy == ZIPNN_RAW || d <= 1) {
            if (lane == 0) {
                EncEntry e;
                e.pad = 0;
                const bool rle = policy != ZIPNN_RAW && d == 1;
                e.mode = rle ? kModeRle : kModeRaw;
                e.rle = rle ? uint8_t(arg) : 0;
                e.bytes = rle ? 0 : m;
                entries[ei] = e;
            }
        } else {
            bool hc = false;
            if (policy != ZIPNN_ZG) {
                uint32_t T;
                hc = build_lengths(fv, m, m, head, p.L, policy == ZIPNN_AUTO, S.pm[k], T);
                if (lane == 0) A.T[0][k] = T;
                if (hc)
#pragma unroll
                    for (int r = 0; r < 4; r++) A.lens[k][lane + 64 * r] = S.pm[k].len[lane + 64 * r];
            }
            const bool zc = policy == ZIPNN_ZG || (policy == ZIPNN_AUTO && 2 * (best >> 8) >= m);
            if (lane == 0) {
                atomicOr(&A.open, 1u << k);
                if (hc) atomicOr(&A.hc, 1u << k);
                if (zc) atomicOr(&A.zc, 1u << k);
                if (zc && ((spec >> k) & 1) && arg == 0) atomicOr(&A.specok, 1u << k);
                A.z[k] = arg;
            }
        }
    }
    __syncthreads();
    // 3. ZG: histogram over the marked groups, then lengths
    if (A.zc) {
        // groups whose ZG histogram the main pass could not give: one more
        // pass over the data
        const uint32_t need = A.zc & ~A.specok;
        if (need) {
            for (uint32_t i = t; i < kWaves * B * 256; i += kBlock) (&S.hist[0][0][0])[i] = 0;
            __syncthreads();
            uint32_t zn[4] = {0, 0, 0, 0};
            switch (p.g) {
            case 2: zg_count<BB, 2>(src, base, need, A.z, m, S.hist[wv], zn, xf); break;
            case 4: zg_count<BB, 4>(src, base, need, A.z, m, S.hist[wv], zn, xf); break;
            default: zg_count<BB, 8>(src, base, need, A.z, m, S.hist[wv], zn, xf); break;
            }
            if (lane == 0)
                for (uint32_t k = 0; k < B; k++) zsum[wv][k] = zn[k];
            __syncthreads();
            for (uint32_t i = t; i < B * 256; i += kBlock) {
                const uint32_t k = i >> 8, s = i & 255;
                uint32_t v = S.hist[0][k][s] + S.hist[1][k][s] + S.hist[2][k][s] + S.hist[3][k][s];
                if (s == A.z[k]) v += zsum[0][k] + zsum[1][k] + zsum[2][k] + zsum[3][k];
                S.hist[0][k][s] = v;
            }
            __syncthreads();
        }
        uint32_t fv[4] = {0, 0, 0, 0}, tot = 0, d2 = 0;
        if (uint32_t(wv) < B) {
            const bool fromspec = (A.specok >> wv) & 1;
            const uint32_t z0 = zspec[0][wv] + zspec[1][wv] + zspec[2][wv] + zspec[3][wv];
#pragma unroll
            for (int r = 0; r < 4; r++) {
                const uint32_t sym = lane + 64 * r;
                fv[r] = fromspec ? (sym == 0 ? z0 : hist[wv][sym]) : S.hist[0][wv][sym];
                tot += fv[r];
                d2 += __popcll(__ballot(fv[r] > 0));
            }
            tot = wave_sum(tot);
        }
        __syncthreads();   // the sums are read before the workspace is reused
        if (uint32_t(wv) < B && ((A.zc >> wv) & 1)) {
            const int k = wv;
            const int policy = A.pol[k];
            if (d2 >= 2) {
                uint32_t T;
                const bool zgc = build_lengths(fv, tot, m, head_z, p.L, policy == ZIPNN_AUTO, S.pm[k], T);
                if (lane == 0) A.T[1][k] = T;
                if (zgc) {
#pragma unroll
                    for (int r = 0; r < 4; r++) A.lens2[k][lane + 64 * r] = S.pm[k].len[lane + 64 * r];
                    if (lane == 0) atomicOr(&A.zgc, 1u << k);
                }
            } else if (policy == ZIPNN_ZG) {
                // the marked groups hold a single value: forced ZG falls back to HUF
                uint32_t f[4];
#pragma unroll
                for (int r = 0; r < 4; r++) f[r] = hist[k][lane + 64 * r];
                uint32_t T;
                build_lengths(f, m, m, head, p.L, false, S.pm[k], T);
#pragma unroll
                for (int r = 0; r < 4; r++) A.lens[k][lane + 64 * r] = S.pm[k].len[lane + 64 * r];
                if (lane == 0) atomicOr(&A.hc, 1u << k);
            }
        }
        __syncthreads();
    }
    // AUTO with both candidates: a candidate that loses even at its best
    // (head + coded bits) against the other at its worst (plus two words
    // of padding per sub-stream) needs no replay; ties go to HUF
    if (uint32_t(t) < B && A.pol[t] == ZIPNN_AUTO && ((A.hc & A.zgc) >> t & 1)) {
        const uint64_t h_lo = head + (A.T[0][t] + 7) / 8, h_hi = h_lo + 8 * W;
        const uint64_t z_lo = head_z + (A.T[1][t] + 7) / 8, z_hi = z_lo + 8 * W;
        if (z_hi < h_lo) atomicAnd(&A.hc, ~(1u << t));
        else if (h_hi <= z_lo) atomicAnd(&A.zgc, ~(1u << t));
    }
    __syncthreads();
    // Staged packing: the packer counts the words, so the sizes are needed
    // here only where the bounds of the candidates (head + coded bits, plus
    // two words of padding per sub-stream) leave AUTO's choice open.
    const bool staged = p.stage != nullptr;
    if (staged && uint32_t(t) < B && ((A.open >> t) & 1) && A.pol[t] == ZIPNN_AUTO) {
        const bool hc = (A.hc >> t) & 1, zgc = (A.zgc >> t) & 1;
        const uint64_t h_lo = head + (A.T[0][t] + 7) / 8, h_hi = h_lo + 8 * W;
        const uint64_t z_lo = head_z + (A.T[1][t] + 7) / 8, z_hi = z_lo + 8 * W;
        bool amb = false;
        uint64_t best_lo = m, best_hi = m;   // RAW
        if (hc) {
            if (h_hi < m) best_lo = h_lo, best_hi = h_hi;
            else if (h_lo < m) amb = true;
        }
        if (zgc && z_hi >= best_lo && z_lo < best_hi) amb = true;
        if (amb) atomicOr(&A.amb, 1u << t);
    }
    __syncthreads();
    const bool exact = !staged || A.amb != 0;
    // 4. the words of every candidate, one lane group per wave
    if ((A.hc | A.zgc) && exact) {
        for (uint32_t j0 = 0; j0 < NG; j0 += kWaves) {
            const uint32_t j = j0 + wv;
            if (j < NG) {
                switch (p.g) {
                case 2: count_lane_group<BB, 2>(src, base, A.hc, A.zgc, A.lens, A.lens2, A.z, p.L, j, W, m, S.lgw, xf); break;
                case 4: count_lane_group<BB, 4>(src, base, A.hc, A.zgc, A.lens, A.lens2, A.z, p.L, j, W, m, S.lgw, xf); break;
                default: count_lane_group<BB, 8>(src, base, A.hc, A.zgc, A.lens, A.lens2, A.z, p.L, j, W, m, S.lgw, xf); break;
                }
                if (lane == 0) {
                    for (uint32_t k = 0; k < B; k++) {
                        if ((A.hc >> k) & 1) atomicAdd(&A.words[0][k], S.lgw[0][k][j]);
                        if ((A.zgc >> k) & 1) atomicAdd(&A.words[1][k], S.lgw[1][k][j]);
                    }
                }
            }
        }
    }
    __syncthreads();
    // 5. the decision, the entry and the word counts of every open group.
    // Without exact sizes (staged, no open choice) the lower bounds decide
    // as the sizes would, and the entry's bytes are left to the packer's
    // counts.
    if (uint32_t(t) < B && ((A.open >> t) & 1)) {
        const int policy = A.pol[t];
        const bool hc = (A.hc >> t) & 1, zgc = (A.zgc >> t) & 1;
        const uint32_t size_h = exact ? head + 4 * A.words[0][t] : head + (A.T[0][t] + 7) / 8;
        const uint32_t size_z = exact ? head_z + 4 * A.words[1][t] : head_z + (A.T[1][t] + 7) / 8;
        int mode = kModeRaw;
        uint32_t bytes = m;
        if (policy == ZIPNN_AUTO) {
            if (hc && size_h < bytes) mode = kModeHuf, bytes = size_h;
            if (zgc && size_z < bytes) mode = kModeZg, bytes = size_z;
        } else if (zgc) {
            mode = kModeZg, bytes = size_z;
        } else {
            mode = kModeHuf, bytes = size_h;
        }
        EncEntry e;
        e.pad = 0;
        e.mode = uint8_t(mode);
        e.rle = mode == kModeZg ? uint8_t(A.z[t]) : 0;
        e.bytes = (staged && mode != kModeRaw) ? 0u : bytes;
        entries[uint64_t(gc) * B + t] = e;
        if (mode != kModeRaw) atomicOr(&A.coded, 1u << t);
        if (mode == kModeZg) atomicOr(&A.fin, 1u << t);
    }
    __syncthreads();
    if (uint32_t(wv) < B && ((A.coded >> wv) & 1)) {
        const uint64_t ei = uint64_t(gc) * B + wv;
        const int v = (A.fin >> wv) & 1;
        canonical_codes(v ? A.lens2[wv] : A.lens[wv], p.L, codes + ei * 256);
        if (!staged && uint32_t(lane) < NG) nwords[ei * 64 + lane] = S.lgw[v][wv][lane];
    }
    __syncthreads();
    return true;
}

// Occupancy matters more than spills here: the passes are latency-bound per
// workgroup.  Four waves per SIMD (128 VGPRs) were 5-9% faster than three;
// for 2-byte words five (96 VGPRs, some spills in the counting loop) encoded
// the BF16 checkpoint 5% and its XOR delta 10% faster than four, and six (80
// VGPRs) are faster again: the checkpoint 1-3% at 256 and 512 KiB chunks, the
// Huffman-only delta 8%.  WV sets the waves per SIMD of the instances for
// 2-byte words.  Where a group of a launch with an XOR base may take ZG, two
// codes are built per group, and seven waves (72 VGPRs) encode the delta 5%
// faster than six (the Huffman-only delta would lose 2%).  Launches with a
// base use these instances only when they take the exact path; staged ones
// run k_analyze_pack.
template <int BB, int WV>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(WV, 8))) void k_analyze(const EncDesc* __restrict__ descs, int n_desc,
                                                    const uint32_t* __restrict__ chunk_prefix, uint32_t total_chunks,
                                                    EncParams p, int phase, EncEntry* __restrict__ entries,
                                                    CodeWord* __restrict__ codes, uint32_t* __restrict__ nwords)
{
    __shared__ AnalyzeShared<BB> sh;
    for (uint32_t gc = blockIdx.x; gc < total_chunks; gc += gridDim.x)
        analyze_chunk<BB>(gc, descs, n_desc, chunk_prefix, p, phase, entries, codes, nwords, sh);
}

// One workgroup per tensor: offsets of its entries (128-byte aligned, in
// chunk-major order) and the tensor's container size.
__global__ __launch_bounds__(kBlock) void k_place(EncDesc* __restrict__ descs, EncParams p,
                                                  EncEntry* __restrict__ entries, uint64_t* __restrict__ offsets,
                                                  uint64_t* __restrict__ totals, const uint32_t* __restrict__ nwords)
{
    __shared__ uint64_t red[kWaves];
    __shared__ uint64_t carry;
    __shared__ uint32_t zg;
    const EncDesc d = descs[blockIdx.x];
    const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
    const uint32_t B = p.B;
    const uint64_t ne = uint64_t(d.n_chunks) * B;
    const uint64_t e_first = uint64_t(d.chunk0) * B;
    if (t == 0) carry = 0, zg = 0;
    __syncthreads();
    for (uint64_t b0 = 0; b0 < ne; b0 += kBlock) {
        const uint64_t e = b0 + t;
        uint64_t sz = 0;
        if (e < ne) {
            EncEntry en = entries[e_first + e];
            if (p.stage && (en.mode == kModeHuf || en.mode == kModeZg)) {
                // staged: the payload's size from the packer's word counts
                const uint32_t E = p.chunk / B;
                const uint32_t m = uint32_t(min(uint64_t(E), d.n - uint64_t(e / B) * E));
                const uint32_t W = (m + p.S - 1) / p.S, NG = (W + 63) / 64;
                uint32_t words = 0;
                for (uint32_t j = 0; j < NG; j++) words += nwords[(e_first + e) * 64 + j];
                en.bytes = huf_head(W) + (en.mode == kModeZg ? zg_bitmap(m, p.g) : 0u) + 4 * words;
                entries[e_first + e].bytes = en.bytes;
            }
            sz = align_pay(en.bytes);
            if (en.mode == kModeZg) zg = 1;
        }
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
        if (e < ne) offsets[e_first + e] = pre + inc - sz;
        __syncthreads();
        if (t == kBlock - 1) carry = pre + inc;
        __syncthreads();
    }
    if (t == 0) {
        totals[blockIdx.x] = payload_base_of(d.n_chunks, B) + carry;
        descs[blockIdx.x].has_zg = zg;
    }
}

// One workgroup: the tensors' containers are laid out back to back in the
// arena (each at a kPayAlign-aligned offset, in tensor order); sets each descriptor's dst,
// writes every header, and records the arena offsets (n+1 of them).  If the
// arena is too small nothing is written and the recorded end says so.
__global__ __launch_bounds__(kBlock) void k_arena(EncDesc* __restrict__ descs, int n_desc, EncParams p,
                                                  uint8_t* __restrict__ arena, uint64_t cap,
                                                  const uint64_t* __restrict__ totals,
                                                  uint64_t* __restrict__ arena_off)
{
    __shared__ uint64_t red[kWaves];
    __shared__ uint64_t carry;
    __shared__ uint64_t end_sh;
    const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
    const uint32_t B = p.B;
    // pass 1: offsets
    if (t == 0) carry = 0;
    __syncthreads();
    for (int b0 = 0; b0 < n_desc; b0 += kBlock) {
        const int i = b0 + t;
        const uint64_t sz = i < n_desc ? align_pay(totals[i]) : 0;
        uint64_t inc = sz;
#pragma unroll
        for (int dd = 1; dd < 64; dd <<= 1) {
            uint64_t o = __shfl_up(inc, dd, 64);
            if (lane >= dd) inc += o;
        }
        if (lane == 63) red[wv] = inc;
        __syncthreads();
        uint64_t pre = carry;
        for (int w = 0; w < wv; w++) pre += red[w];
        if (i < n_desc) arena_off[i] = pre + inc - sz;
        __syncthreads();
        if (t == kBlock - 1) carry = pre + inc;
        __syncthreads();
    }
    if (t == 0) {
        // the last container needs only its own bytes, not the alignment
        end_sh = n_desc ? arena_off[n_desc - 1] + totals[n_desc - 1] : 0;
        arena_off[n_desc] = end_sh;
    }
    __syncthreads();
    const bool fits = end_sh <= cap;
    for (int i = t; i < n_desc; i += kBlock) {
        EncDesc d = descs[i];
        d.dst = arena + arena_off[i];
        d.dst_cap = fits ? totals[i] : 0;   // pack skips tensors whose dst_cap is short
        descs[i] = d;
        if (!fits) continue;
        const uint64_t total = totals[i];
        uint32_t h[16];
        h[0] = 0x314E4E5Au;
        h[1] = 1u | (p.dtype << 16) | (B << 24);
        h[2] = uint32_t(d.n);
        h[3] = uint32_t(d.n >> 32);
        h[4] = p.chunk;
        h[5] = p.S | (p.g << 16) | (p.L << 24);
        h[6] = (d.base ? kFlagDelta : 0u) | (d.has_zg ? kFlagZg : 0u) | (p.flags & kFlagExp);
        h[7] = d.n_chunks;
        h[8] = uint32_t(total);
        h[9] = uint32_t(total >> 32);
        h[10] = 0;
        for (uint32_t k = 0; k < B; k++) h[10] |= uint32_t(p.policy[k]) << (8 * k);
        h[11] = p.skip;   // byte 44: the probe interval
        for (int x = 12; x < 16; x++) h[x] = 0;
        uint4* o = (uint4*)d.dst;
        for (int x = 0; x < 4; x++) o[x] = make_uint4(h[4 * x], h[4 * x + 1], h[4 * x + 2], h[4 * x + 3]);
        // zero padding between the map and the aligned payload area
        const uint64_t map_end = 64 + 16ull * d.n_chunks * B, pb = payload_base_of(d.n_chunks, B);
        for (uint64_t x = map_end / 16; x < pb / 16; x++) o[x] = make_uint4(0, 0, 0, 0);
    }
}

struct PackLds {
    uint32_t rcode[4][256];     // reversed code | length << 27 (0 for absent symbols)
    uint64_t pay[4];            // absolute payload offset of each stream
    uint32_t mode[4];
    uint32_t bytes[4];
    uint32_t z[4];              // ZG fill value
    uint32_t wpre[4][65];       // lane-group word prefix per stream
};

constexpr uint32_t kLenShift = 27;              // code length's place in a packer code entry

// f(integral_constant<int, k>) for k = 0 .. N-1: per-stream state is then
// picked at compile time and stays in registers
template <int N, class F>
__device__ __attribute__((always_inline)) inline void for_streams(F&& f)
{
    if constexpr (N > 0) {
        for_streams<N - 1>(f);
        f(std::integral_constant<int, N - 1>{});
    }
}
constexpr uint32_t kNoStore = 0x80000000u;      // buffer offset past every resource: the store is dropped

// Write the words of lane group j of every coded stream of one chunk (bit k
// of cm; with bit k of zm a ZG stream with fill value P.z[k], whose unmarked
// groups are not coded) in one pass over the chunk's groups, in lock-step
// over the steps and pairs of the layout.  Per stream, at every pair of its
// coded groups a lane first takes a word if it holds fewer than 2L bits: the
// word's place is the lane group's cursor plus the lane's rank among the
// pair's takers.  Then the pair's codes join the lane's bits, and a word that
// is complete is stored at the oldest place taken for it.  With held =
// 32 * taken - consumed and nacc the coded bits not yet stored, held + nacc is
// 32 times the words taken and not yet stored: a taken word lies wholly past
// what the lane has consumed, so it is finished later, and at most two are
// ever unfinished (after each take held lies in [2L, 2L + 31]).  After the
// lane's last pair the unfinished words are stored: the partial one, then
// zero.  The stores go through a buffer resource over the lane group's words,
// so a place past them (which the analysis's counts never give) is dropped.
// Steps in which every lane has a full group run without per-lane group
// counts; the raw byte groups of small groups are copied on the same pass.
// Staged (stage_lg > 0): stream k's payload area is the staging slot at
// P.pay[k], lane group j's words start at stage_bm + j * stage_lg, a ZG
// bitmap at the slot's start; the lane group's word count goes to
// nw_out[k * 64 + j].
template <int B, int G>
__device__ __attribute__((always_inline)) void pack_lane_group(const uint8_t* src, const uint8_t* base, uint32_t cm,
                                                               uint32_t zm, const PackLds& P, uint32_t L, uint32_t j,
                                                               uint32_t W, uint32_t m, bool xf, bool fuse_bitmap,
                                                               uint32_t rawmask, uint8_t* dst, uint32_t stage_lg,
                                                               uint32_t stage_bm, uint32_t* nw_out)
{
    constexpr int NB = B * G;
    constexpr int NW = NB >= 4 ? NB / 4 : 1;
    // groups of input prefetched ahead (two for 4-byte words: fewer registers)
    constexpr uint32_t kPf = B == 4 ? 2 : 4;
    cm = __builtin_amdgcn_readfirstlane(cm);
    zm = __builtin_amdgcn_readfirstlane(zm);
    // the lane group is the wave's: uniform, so every value derived from it
    // (a buffer resource above all) stays in scalar registers
    j = __builtin_amdgcn_readfirstlane(j);
    const uint32_t lane = threadIdx.x & 63;
    const uint32_t w = 64 * j + lane;
    const int twoL = int(2 * L);
    const uint32_t Gtot = (m + G - 1) / G, Gfull = m / G, rem = m - Gfull * G;
    const uint32_t ng = (w < W && w < Gtot) ? (Gtot - 1 - w) / W + 1 : 0;
    const uint32_t ng_max = __builtin_amdgcn_readfirstlane(ng);   // lane 0 has the most
    // full groups of the lane group's last lane: every lane has at least these
    const uint32_t w_last = min(W, 64 * j + 64) - 1;
    const uint32_t nfull_all = w_last < Gfull ? (Gfull - 1 - w_last) / W + 1 : 0;
    const uint32_t n_fast = (64 * j + 64 <= W) ? nfull_all / kPf * kPf : 0;
    const uint32_t head = huf_head(W), bm = zg_bitmap(m, G);
    auto uni64 = [](uint64_t v) {
        return uint64_t(uint32_t(__builtin_amdgcn_readfirstlane(uint32_t(v)))) |
               (uint64_t(uint32_t(__builtin_amdgcn_readfirstlane(uint32_t(v >> 32)))) << 32);
    };
    // per coded stream: its words of this lane group (a buffer resource), the
    // fused bitmap, and the lock-step state
    struct Stream {
        __amdgpu_buffer_rsrc_t out;
        uint64_t* bmw;
        uint32_t cur, alo, ahi, nacc, s0, s1;
        int held;
    };
    Stream st0, st1, st2, st3;
    auto S = [&](auto kc) __attribute__((always_inline)) -> Stream& {
        constexpr int k = decltype(kc)::value;
        if constexpr (k == 0) return st0;
        else if constexpr (k == 1) return st1;
        else if constexpr (k == 2) return st2;
        else return st3;
    };
    for_streams<B>([&](auto kc) __attribute__((always_inline)) {
        constexpr int k = decltype(kc)::value;
        Stream& x = S(kc);
        const uint32_t zb = (zm >> k) & 1;
        const uint64_t pk = uni64(P.pay[k]);
        const bool staged = stage_lg != 0;
        const uint32_t w0 = staged ? j * (stage_lg / 4) : __builtin_amdgcn_readfirstlane(P.wpre[k][j]);
        const uint32_t nw = staged ? stage_lg / 4 : __builtin_amdgcn_readfirstlane(P.wpre[k][j + 1]) - w0;
        const uint32_t lead = staged ? stage_bm : head + (zb ? bm : 0u);   // bytes before the words
        const uint64_t wa = uni64(uint64_t(dst + pk + lead) + 4ull * w0);
        x.out = __builtin_amdgcn_make_buffer_rsrc(reinterpret_cast<void*>(wa), (short)0,
                                                  int(((cm >> k) & 1) ? 4 * nw : 0u), 0x00020000);
        x.bmw = (zb && fuse_bitmap) ? reinterpret_cast<uint64_t*>(dst + pk + (staged ? 0u : head)) : nullptr;
        x.cur = x.alo = x.ahi = x.nacc = x.s0 = x.s1 = 0;
        x.held = 0;
    });
    // raw byte groups copied here (groups of at most 4 bytes: b16 / b32
    // stores through one resource over the chunk's payloads, which are
    // consecutive, and a scalar offset per raw group)
    constexpr bool kFuseRaw = G <= 4 && B * G <= 16;
    const uint64_t raw0 = uni64(uint64_t(dst + P.pay[0]));
    const __amdgpu_buffer_rsrc_t rr = __builtin_amdgcn_make_buffer_rsrc(
        reinterpret_cast<void*>(raw0), (short)0,
        int(__builtin_amdgcn_readfirstlane(rawmask ? uint32_t(P.pay[B - 1] - P.pay[0]) + m : 0u)), 0x00020000);
    // one pair of stream k: entries c0, c1 (zero for a symbol that is not
    // coded), p0 whether the lane takes part
    auto pair = [&](auto kc, uint32_t c0, uint32_t c1, bool p0) __attribute__((always_inline)) {
        Stream& x = S(kc);
        const bool need = p0 && x.held < twoL;
        const uint64_t msk = __ballot(need);
        const uint32_t rank =
            __builtin_amdgcn_mbcnt_hi(uint32_t(msk >> 32), __builtin_amdgcn_mbcnt_lo(uint32_t(msk), 0u));
        const uint32_t place = (x.cur + rank) * 4u;
        // nothing pending: held + nacc = 0, i.e. held = 0 (nacc < 32)
        const bool empty = x.held == 0;
        x.s0 = (need && empty) ? place : x.s0;
        x.s1 = need ? place : x.s1;
        x.held += need ? 32 : 0;
        x.cur += uint32_t(__popcll(msk));
        // the two codes side by side (the lengths sit in bits 27..31 of an
        // entry, so the entries' sum carries the sum of the lengths, <= 2L)
        const uint32_t l0 = c0 >> kLenShift, l = (c0 + c1) >> kLenShift;
        const uint32_t pc = (c0 | (c1 << l0)) & ((1u << kLenShift) - 1);
        const uint64_t v = uint64_t(pc) << x.nacc;
        x.alo |= uint32_t(v);
        x.ahi |= uint32_t(v >> 32);
        x.nacc += l;
        x.held -= int(l);
        // at most one word completes per pair (nacc < 32 + 2L)
        const bool full = x.nacc >= 32;
        __builtin_amdgcn_raw_buffer_store_b32(x.alo, x.out, full ? x.s0 : kNoStore, 0, 0);
        x.alo = full ? x.ahi : x.alo;
        x.ahi = 0;   // fewer than 32 bits left: none above the low word
        x.nacc &= 31u;
        x.s0 = full ? x.s1 : x.s0;
    };
    // one step (group e of every lane); FAST: every lane has a full group
    auto step = [&](uint32_t e, const uint32_t* wd, auto fast_c) __attribute__((always_inline)) {
        constexpr bool FAST = decltype(fast_c)::value;
        const bool has = FAST || e < ng;
        const uint32_t ecnt = FAST ? uint32_t(G) : (has ? (w + e * W < Gfull ? G : rem) : 0u);
        if constexpr (kFuseRaw) {
            if (rawmask && has) {
                const uint32_t q0 = (w + e * W) * G;
                for_streams<B>([&](auto rc) __attribute__((always_inline)) {
                    constexpr int r = decltype(rc)::value;
                    if (!((rawmask >> r) & 1)) return;
                    const uint32_t roff = __builtin_amdgcn_readfirstlane(uint32_t(P.pay[r] - P.pay[0]));
                    if (FAST || ecnt == G) {
                        const uint32_t v = gather_stream<B, G>(wd, r);
                        if constexpr (G == 2) __builtin_amdgcn_raw_buffer_store_b16(uint16_t(v), rr, q0, roff, 0);
                        else __builtin_amdgcn_raw_buffer_store_b32(v, rr, q0, roff, 0);
                    } else {
                        for (uint32_t i = 0; i < ecnt; i++)
                            __builtin_amdgcn_raw_buffer_store_b8(uint8_t(sym_of<B>(wd, r, int(i))), rr, q0 + i, roff,
                                                                 0);
                    }
                });
            }
        }
        for_streams<B>([&](auto kc) __attribute__((always_inline)) {
            constexpr int k = decltype(kc)::value;
            if (!((cm >> k) & 1)) return;
            // the pairs of a group of gcnt coded symbols
            auto pairs = [&](uint32_t gcnt) __attribute__((always_inline)) {
#pragma unroll
                for (int pr = 0; pr < G / 2; pr++) {
                    const bool p0 = 2u * pr < gcnt, p1 = 2u * pr + 1 < gcnt;
                    const uint32_t c0 = P.rcode[k][sym_of<B>(wd, k, 2 * pr)];
                    const uint32_t c1 = P.rcode[k][sym_of<B>(wd, k, 2 * pr + 1)];
                    pair(kc, p0 ? c0 : 0u, p1 ? c1 : 0u, p0);
                }
            };
            if ((zm >> k) & 1) {
                const bool mk = has && marked<B, G>(wd, k, ecnt, P.z[k]);
                const uint64_t bits = __ballot(mk);
                // ZG with W a multiple of 64: the 64 bits of this lane
                // group's step e are one aligned word of the bitmap
                if (fuse_bitmap && lane == 0) S(kc).bmw[j + e * (W / 64)] = bits;
                // where no lane of the wave holds a marked group, the pairs
                // would take no word and add no bits: they are skipped
                if (bits) pairs(mk ? ecnt : 0u);
            } else {
                pairs(ecnt);   // in a fast step, G: no per-lane conditions
            }
        });
    };
    auto load = [&](uint32_t e, uint32_t* wd) {
        if (e < ng) group_words<B, G>(src, base, w + e * W, m, wd, xf);
    };
    uint32_t pf[kPf][NW];
#pragma unroll
    for (uint32_t u = 0; u < kPf; u++) load(u, pf[u]);
    for (uint32_t j0 = 0; j0 < n_fast; j0 += kPf) {
#pragma unroll
        for (uint32_t u = 0; u < kPf; u++) {
            uint32_t cw[NW];
#pragma unroll
            for (int x = 0; x < NW; x++) cw[x] = pf[u][x];
            load(j0 + u + kPf, pf[u]);
            step(j0 + u, cw, std::integral_constant<bool, true>{});
        }
    }
    for (uint32_t j0 = n_fast; j0 < ng_max; j0 += kPf) {
#pragma unroll
        for (uint32_t u = 0; u < kPf; u++) {
            const uint32_t jj = j0 + u;
            if (jj < ng_max) {
                uint32_t cw[NW];
#pragma unroll
                for (int x = 0; x < NW; x++) cw[x] = pf[u][x];
                load(jj + kPf, pf[u]);
                step(jj, cw, std::integral_constant<bool, false>{});
            }
        }
    }
    // the lane's unfinished words: the partial one (zero bits if none), then zero
    for_streams<B>([&](auto kc) __attribute__((always_inline)) {
        constexpr int k = decltype(kc)::value;
        if (!((cm >> k) & 1)) return;
        const Stream& x = S(kc);
        const int pend = (x.held + int(x.nacc)) >> 5;
        __builtin_amdgcn_raw_buffer_store_b32(x.alo, x.out, pend > 0 ? x.s0 : kNoStore, 0, 0);
        __builtin_amdgcn_raw_buffer_store_b32(0u, x.out, pend > 1 ? x.s1 : kNoStore, 0, 0);
        // staged: the words this lane group took (the cursor is uniform)
        if (nw_out && lane == 0) nw_out[k * 64 + j] = x.cur;
    });
}

// The group bitmap of a ZG stream: wave v writes 64-bit words x = v, v+4, ...
// of the bm bytes (lane l tests group 64x + l); bits past the last group and
// the padding are zero.
template <int B, int G>
__device__ void pack_bitmap(const uint8_t* src, const uint8_t* base, int k, uint32_t z, uint32_t m, uint32_t bm,
                            uint8_t* dst, bool xf)
{
    constexpr int NB = B * G;
    constexpr int NW = NB >= 4 ? NB / 4 : 1;
    const uint32_t lane = threadIdx.x & 63;
    const uint32_t Gtot = (m + G - 1) / G;
    for (uint32_t x = threadIdx.x >> 6; x < bm / 8; x += kWaves) {
        const uint32_t q = 64 * x + lane;
        bool mk = false;
        if (q < Gtot) {
            uint32_t wd[NW];
            group_words<B, G>(src, base, q, m, wd, xf);
            mk = marked<B, G>(wd, k, min(uint32_t(G), m - q * G), z);
        }
        const uint64_t bits = __ballot(mk);
        if (lane == 0) *reinterpret_cast<uint64_t*>(dst + 8 * x) = bits;
    }
}

// Raw groups of one chunk: thread t copies elements [16u, 16u+16) of every
// RAW stream with one 16-byte store each, then the zero padding.  With
// pad_only the packer of a coded group copies the elements, and only the
// padding is written here.
template <int B>
__device__ void pack_raw(const uint8_t* src, const uint8_t* base, uint8_t* dst, const PackLds& P, uint32_t m, bool xf,
                         bool pad_only)
{
    uint32_t rawmask = 0;
    for (int k = 0; k < B; k++)
        if (P.mode[k] == kModeRaw) rawmask |= 1u << k;
    if (!rawmask) return;
    if (pad_only) {
        for (uint32_t e = m + threadIdx.x; e < uint32_t(align_pay(m)); e += kBlock)
#pragma unroll
            for (int k = 0; k < B; k++)
                if ((rawmask >> k) & 1) dst[P.pay[k] + e] = 0;
        return;
    }
    const uint32_t units = m / 16;
    constexpr uint32_t RB = B == 4 ? 2 : (B == 2 ? 4 : 8);   // units in flight per thread
    for (uint32_t u0 = threadIdx.x; u0 < units; u0 += RB * kBlock) {
        uint32_t wds[RB][4 * B];
#pragma unroll
        for (uint32_t r = 0; r < RB; r++) {
            const uint32_t u = u0 + r * kBlock;
            if (u < units) {
                loadNB<16 * B>(src + uint64_t(u) * 16 * B, wds[r]);
                if (base) {
                    uint32_t bw[4 * B];
                    loadNB<16 * B>(base + uint64_t(u) * 16 * B, bw);
#pragma unroll
                    for (int x = 0; x < 4 * B; x++) wds[r][x] ^= bw[x];
                }
                if (xf)
#pragma unroll
                    for (int x = 0; x < 4 * B; x++) wds[r][x] = exp_fwd<B>(wds[r][x]);
            }
        }
#pragma unroll
        for (uint32_t r = 0; r < RB; r++) {
            const uint32_t u = u0 + r * kBlock;
#pragma unroll
            for (int k = 0; k < B; k++) {
                if (!((rawmask >> k) & 1) || u >= units) continue;
                uint32_t o[4] = {0, 0, 0, 0};
#pragma unroll
                for (int i = 0; i < 16; i++) o[i >> 2] |= sym_of<B>(wds[r], k, i) << (8 * (i & 3));
                *(uint4*)(dst + P.pay[k] + 16 * u) = make_uint4(o[0], o[1], o[2], o[3]);
            }
        }
    }
    // tail elements, then zero padding to the payload alignment
    for (uint32_t e = units * 16 + threadIdx.x; e < uint32_t(align_pay(m)); e += kBlock) {
        const uint32_t v = e < m ? element_word<B>(src, base, e, xf) : 0u;
#pragma unroll
        for (int k = 0; k < B; k++)
            if ((rawmask >> k) & 1) dst[P.pay[k] + e] = uint8_t(v >> (8 * (B - 1 - k)));
    }
}

// Five waves per SIMD for 2-byte words (at most 96 VGPRs, a few spills
// outside the pair loop: the BF16 deltas' encode 6% faster, the checkpoint's
// unchanged), four for the others (at most 128; the FP32 g = 4 instance
// spills).  XB: the instance for launches with an XOR base, six waves for
// 2-byte words (80 VGPRs): the deltas 4% faster again, where the plain
// checkpoint would lose 2%.
// The packing of chunk gc by one workgroup (into its container, or staged
// into its staging slots with the word counts).
template <int BB, int GG>
__device__ __attribute__((always_inline)) void pack_chunk(uint32_t gc, const EncDesc* __restrict__ descs, int n_desc,
                                                          const uint32_t* __restrict__ chunk_prefix, const EncParams& p,
                                                          const EncEntry* __restrict__ entries,
                                                          const CodeWord* __restrict__ codes,
                                                          const uint64_t* __restrict__ offsets,
                                                          const uint64_t* __restrict__ totals,
                                                          uint32_t* __restrict__ nwords, PackLds& P)
{
    const int t = threadIdx.x, wv = t >> 6;
    constexpr uint32_t B = BB;
    // staged: the payloads go to the staging slots (their places in the
    // container are not known yet) and the word counts come out
    const bool staged = p.stage != nullptr;
    const int di = find_desc(chunk_prefix, n_desc, gc);
    const EncDesc d = descs[di];
    if (!staged && totals[di] > d.dst_cap) return;   // too small: the host reports it
    const uint32_t c = gc - chunk_prefix[di];
    const uint32_t E = p.chunk / B;
    const uint64_t e0 = uint64_t(c) * E;
    const uint32_t m = uint32_t(min(uint64_t(E), d.n - e0));
    const uint32_t W = (m + p.S - 1) / p.S;
    const uint32_t NG = (W + 63) / 64;
    const uint32_t head = huf_head(W);
    const uint64_t payload_base = payload_base_of(d.n_chunks, B);
    for (uint32_t k = 0; k < B; k++) {
        const uint64_t ei = uint64_t(gc) * B + k;
        const EncEntry en = entries[ei];
        if (t == 0 && staged) {
            P.mode[k] = en.mode;
            P.bytes[k] = en.bytes;
            P.pay[k] = ei * p.stage_chunk;
        } else if (t == 0) {
            P.mode[k] = en.mode;
            P.bytes[k] = en.bytes;
            P.pay[k] = payload_base + offsets[ei];
            // this chunk's map entry
            uint4 ent;
            ent.x = uint32_t(offsets[ei]);
            ent.y = uint32_t(offsets[ei] >> 32);
            ent.z = en.bytes;
            ent.w = uint32_t(en.mode) | (uint32_t(en.rle) << 8);
            *(uint4*)(d.dst + 64 + 16 * (uint64_t(c) * B + k)) = ent;
        }
        if (t == 0) P.z[k] = en.rle;
        if (en.mode == kModeHuf || en.mode == kModeZg) {
            const uint32_t cw = codes[ei * 256 + t];
            const uint32_t l = cw >> 16;
            P.rcode[k][t] = l ? ((__brev(cw & 0xFFFFu) >> (32 - l)) | (l << kLenShift)) : 0u;
            if (t < 64 && !staged) {
                const uint32_t nw = uint32_t(t) < NG ? nwords[ei * 64 + t] : 0u;
                uint32_t inc = nw;
#pragma unroll
                for (int dd = 1; dd < 64; dd <<= 1) {
                    uint32_t o = __shfl_up(inc, dd, 64);
                    if (t >= dd) inc += o;
                }
                P.wpre[k][t + 1] = inc;
                if (t == 0) P.wpre[k][0] = 0;
            }
        }
    }
    __syncthreads();
    const uint8_t* src = d.src + e0 * B;
    const uint8_t* base = d.base ? d.base + e0 * B : nullptr;
    uint8_t* dst = staged ? p.stage : d.dst;
    const bool xf = (p.flags & kFlagExp) != 0;
    // the coded groups (HUF and ZG) are packed in one pass, which also
    // copies the raw groups when groups are small (at most 4 bytes)
    uint32_t rawmask = 0, cm = 0, zm = 0;
    for (uint32_t k = 0; k < B; k++) {
        if (P.mode[k] == kModeRaw) rawmask |= 1u << k;
        if (P.mode[k] == kModeHuf || P.mode[k] == kModeZg) cm |= 1u << k;
        if (P.mode[k] == kModeZg) zm |= 1u << k;
    }
    const bool fuse_raw = GG <= 4 && BB * GG <= 16 && cm != 0;
    pack_raw<BB>(src, base, dst, P, m, xf, fuse_raw);
    // with W a multiple of 64 the packer writes a ZG bitmap's words as it
    // marks the groups
    const bool fuse_bitmap = W % 64 == 0;
    for (uint32_t k = 0; k < B; k++) {
        const bool zg = P.mode[k] == kModeZg;
        if (P.mode[k] != kModeHuf && !zg) continue;
        uint8_t* pay = dst + P.pay[k];
        // head: nibble table, word counts, zero pad; ZG bitmap; zero pad
        // after words (staged: the compaction writes all but the bitmap)
        if (!staged) {
            if (t < 128)
                pay[t] = uint8_t((P.rcode[k][2 * t] >> kLenShift) | ((P.rcode[k][2 * t + 1] >> kLenShift) << 4));
            if (uint32_t(t) < NG) ((uint32_t*)(pay + 128))[t] = P.wpre[k][t + 1] - P.wpre[k][t];
            for (uint32_t i = 128 + 4 * NG + t; i < head; i += kBlock) pay[i] = 0;
            for (uint32_t i = P.bytes[k] + t; i < uint32_t(align_pay(P.bytes[k])); i += kBlock) pay[i] = 0;
        }
        const uint32_t lead = staged ? 0u : head;   // where the bitmap starts
        if (zg) {
            const uint32_t bm = zg_bitmap(m, GG);
            if (fuse_bitmap) {   // only the words past the last group are zeroed here
                uint64_t* words = reinterpret_cast<uint64_t*>(pay + lead);
                const uint32_t Gtot = (m + GG - 1) / GG;
                for (uint32_t x = (Gtot + 63) / 64 + t; x < bm / 8; x += kBlock) words[x] = 0;
            } else {
                pack_bitmap<BB, GG>(src, base, int(k), P.z[k], m, bm, pay + lead, xf);
            }
        }
    }
    if (cm)
        for (uint32_t j = wv; j < NG; j += kWaves)
            pack_lane_group<BB, GG>(src, base, cm, zm, P, p.L, j, W, m, xf, fuse_bitmap, fuse_raw ? rawmask : 0u,
                                    dst, staged ? p.stage_lg : 0u, p.stage_bm,
                                    staged ? nwords + uint64_t(gc) * B * 64 : nullptr);
    __syncthreads();
}

template <int BB, int GG, bool XB>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(BB == 2 ? (XB ? 6 : 5) : 4, 8))) void k_pack(const EncDesc* __restrict__ descs, int n_desc,
                                                 const uint32_t* __restrict__ chunk_prefix, uint32_t total_chunks,
                                                 EncParams p, const EncEntry* __restrict__ entries,
                                                 const CodeWord* __restrict__ codes,
                                                 const uint64_t* __restrict__ offsets,
                                                 const uint64_t* __restrict__ totals,
                                                 uint32_t* __restrict__ nwords)
{
    __shared__ PackLds P;
    for (uint32_t gc = blockIdx.x; gc < total_chunks; gc += gridDim.x)
        pack_chunk<BB, GG>(gc, descs, n_desc, chunk_prefix, p, entries, codes, offsets, totals, nwords, P);
}

template <int BB>
union FusedLds {
    AnalyzeShared<BB> a;
    PackLds pk;
};

// Staged launches: a workgroup analyses a chunk and packs it at once into its
// staging slots, which need no placement first; a chunk's analysis and
// packing thus share a launch, and the workgroups on a CU mix the two (the
// checkpoint's XOR delta: Huffman-only encode 16.9 -> 16.0 ms, zero-aware
// 18.4 -> 17.5 ms).  For 2-byte words seven waves per SIMD (72 VGPRs):
// faster than six by 5% on the Huffman-only delta, and by about 10% than
// five.
template <int BB, int GG, int WV>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(WV, 8))) void k_analyze_pack(
    const EncDesc* __restrict__ descs, int n_desc, const uint32_t* __restrict__ chunk_prefix, uint32_t total_chunks,
    EncParams p, int phase, EncEntry* entries, CodeWord* codes, uint32_t* nwords)
{
    __shared__ FusedLds<BB> u;
    for (uint32_t gc = blockIdx.x; gc < total_chunks; gc += gridDim.x) {
        if (!analyze_chunk<BB>(gc, descs, n_desc, chunk_prefix, p, phase, entries, codes, nwords, u.a)) continue;
        __syncthreads();   // the chunk's entries and code tables, written above, are read below
        pack_chunk<BB, GG>(gc, descs, n_desc, chunk_prefix, p, entries, codes, nullptr, nullptr, nwords, u.pk);
        __syncthreads();
    }
}

// Staged packing, last step: for each chunk, its map entries, and for each
// coded stream the head (nibble table, word counts, padding), the ZG bitmap
// and the lane groups' words copied from their staging slots to their places;
// raw streams are copied whole; then the zero padding to the payload
// alignment.  Tensors whose container did not fit the arena are skipped.
template <int BB, int GG>
__global__ __launch_bounds__(kBlock) void k_compact(const EncDesc* __restrict__ descs, int n_desc,
                                                    const uint32_t* __restrict__ chunk_prefix, uint32_t total_chunks,
                                                    EncParams p, const EncEntry* __restrict__ entries,
                                                    const CodeWord* __restrict__ codes,
                                                    const uint64_t* __restrict__ offsets,
                                                    const uint64_t* __restrict__ totals,
                                                    const uint32_t* __restrict__ nwords)
{
    __shared__ uint32_t wpre[65];
    const int t = threadIdx.x;
    constexpr uint32_t B = BB;
    for (uint32_t gc = blockIdx.x; gc < total_chunks; gc += gridDim.x) {
        const int di = find_desc(chunk_prefix, n_desc, gc);
        const EncDesc d = descs[di];
        if (totals[di] > d.dst_cap) continue;   // too small: the host reports it
        const uint32_t c = gc - chunk_prefix[di];
        const uint32_t E = p.chunk / B;
        const uint32_t m = uint32_t(min(uint64_t(E), d.n - uint64_t(c) * E));
        const uint32_t W = (m + p.S - 1) / p.S;
        const uint32_t NG = (W + 63) / 64;
        const uint32_t head = huf_head(W);
        const uint64_t payload_base = payload_base_of(d.n_chunks, B);
        for (uint32_t k = 0; k < B; k++) {
            const uint64_t ei = uint64_t(gc) * B + k;
            const EncEntry en = entries[ei];
            if (t == 0) {
                uint4 ent;
                ent.x = uint32_t(offsets[ei]);
                ent.y = uint32_t(offsets[ei] >> 32);
                ent.z = en.bytes;
                ent.w = uint32_t(en.mode) | (uint32_t(en.rle) << 8);
                *(uint4*)(d.dst + 64 + 16 * (uint64_t(c) * B + k)) = ent;
            }
            uint8_t* pay = d.dst + payload_base + offsets[ei];
            const uint8_t* slot = p.stage + ei * p.stage_chunk;
            if (en.mode == kModeRaw) {
                // 16-byte pieces (both ends are 16-byte aligned), then the tail
                for (uint32_t i = t; i < m / 16; i += kBlock)
                    reinterpret_cast<uint4*>(pay)[i] = reinterpret_cast<const uint4*>(slot)[i];
                for (uint32_t i = m / 16 * 16 + t; i < m; i += kBlock) pay[i] = slot[i];
            } else if (en.mode == kModeHuf || en.mode == kModeZg) {
                const bool zg = en.mode == kModeZg;
                const uint32_t bm = zg ? zg_bitmap(m, GG) : 0u;
                if (t < 128)
                    pay[t] = uint8_t((codes[ei * 256 + 2 * t] >> 16) | ((codes[ei * 256 + 2 * t + 1] >> 16) << 4));
                if (t < 64) {
                    const uint32_t nw = uint32_t(t) < NG ? nwords[ei * 64 + t] : 0u;
                    if (uint32_t(t) < NG) reinterpret_cast<uint32_t*>(pay + 128)[t] = nw;
                    uint32_t inc = nw;
#pragma unroll
                    for (int dd = 1; dd < 64; dd <<= 1) {
                        uint32_t o = __shfl_up(inc, dd, 64);
                        if (t >= dd) inc += o;
                    }
                    wpre[t + 1] = inc;
                    if (t == 0) wpre[0] = 0;
                }
                for (uint32_t i = 128 + 4 * NG + t; i < head; i += kBlock) pay[i] = 0;
                for (uint32_t i = t; i < bm / 16; i += kBlock)
                    reinterpret_cast<uint4*>(pay + head)[i] = reinterpret_cast<const uint4*>(slot)[i];
                __syncthreads();
                uint32_t* words = reinterpret_cast<uint32_t*>(pay + head + bm);
                for (uint32_t j = 0; j < NG; j++) {
                    const uint32_t* from = reinterpret_cast<const uint32_t*>(slot + p.stage_bm + uint64_t(j) * p.stage_lg);
                    const uint32_t w0 = wpre[j], nw = wpre[j + 1] - w0;
                    for (uint32_t i = t; i < nw; i += kBlock) words[w0 + i] = from[i];
                }
            }
            for (uint32_t i = en.bytes + t; i < uint32_t(align_pay(en.bytes)); i += kBlock) pay[i] = 0;
            __syncthreads();
        }
    }
}

// One tensor's descriptor and chunk prefix, written from kernel arguments (the
// allocation-free entry point has no host staging to copy them from).
__global__ void k_fill_desc(EncDesc one, uint32_t total_chunks, EncDesc* __restrict__ d, uint32_t* __restrict__ prefix)
{
    if (threadIdx.x == 0) {
        *d = one;
        prefix[0] = 0;
        prefix[1] = total_chunks;
    }
}

}  // namespace

hipError_t launch_fill_desc(const EncDesc& one, uint32_t total_chunks, EncDesc* d_desc, uint32_t* d_prefix,
                            hipStream_t s)
{
    k_fill_desc<<<1, 64, 0, s>>>(one, total_chunks, d_desc, d_prefix);
    return hipGetLastError();
}

hipError_t launch_encode(EncDesc* d_descs, int n_desc, const uint32_t* d_chunk_prefix, uint32_t total_chunks,
                         const EncParams& p, uint8_t* arena, uint64_t cap, EncEntry* entries, CodeWord* codes,
                         uint32_t* nwords, uint64_t* offsets, uint64_t* totals, uint64_t* arena_off, hipStream_t s)
{
    const uint32_t grid = min(max(total_chunks, 1u), 1u << 16);
    const bool xb = (p.flags & kFlagDelta) != 0;   // some tensor has an XOR base
    bool zg_possible = false;                       // some group may take ZG
    for (uint32_t k = 0; k < p.B && k < 4; k++) zg_possible |= p.policy[k] == ZIPNN_AUTO || p.policy[k] == ZIPNN_ZG;
    const bool staged = p.stage != nullptr;
    if (total_chunks) {
        // with probing, the probe chunks first: the others read their entries
        for (int phase = p.skip ? 0 : -1; phase <= (p.skip ? 1 : -1); phase++) {
            bool launched = false;
            if (staged) {
#define ZIPNN_FUSED(B_, G_, WV_)                                                                                 \
    if (!launched && p.B == B_ && p.g == G_) {                                                                  \
        k_analyze_pack<B_, G_, WV_><<<grid, kBlock, 0, s>>>(d_descs, n_desc, d_chunk_prefix, total_chunks, p,   \
                                                            phase, entries, codes, nwords);                      \
        launched = true;                                                                                        \
    }
                ZIPNN_FUSED(1, 2, 4) ZIPNN_FUSED(1, 4, 4) ZIPNN_FUSED(1, 8, 4)
                ZIPNN_FUSED(2, 2, 7) ZIPNN_FUSED(2, 4, 7) ZIPNN_FUSED(2, 8, 7)
                ZIPNN_FUSED(4, 2, 4) ZIPNN_FUSED(4, 4, 4) ZIPNN_FUSED(4, 8, 4)
#undef ZIPNN_FUSED
            } else {
#define ZIPNN_ANALYZE(B_, WV_)                                                                                   \
    k_analyze<B_, WV_><<<grid, kBlock, 0, s>>>(d_descs, n_desc, d_chunk_prefix, total_chunks, p, phase, entries, \
                                               codes, nwords)
                launched = true;
                if (p.B == 1) ZIPNN_ANALYZE(1, 4);
                else if (p.B == 2 && xb && zg_possible) ZIPNN_ANALYZE(2, 7);
                else if (p.B == 2) ZIPNN_ANALYZE(2, 6);
                else if (p.B == 4) ZIPNN_ANALYZE(4, 4);
                else launched = false;
#undef ZIPNN_ANALYZE
            }
            if (!launched) return hipErrorInvalidValue;
            if (hipGetLastError() != hipSuccess) return hipErrorLaunchFailure;
        }
    }
    // exact: analysis, placement, arena, then packing into the containers;
    // staged: analysis with packing into the staging slots, placement from
    // the word counts, arena, then the compaction into the containers
    auto pack_or_compact = [&](bool compact) -> hipError_t {
        if (!total_chunks) return hipSuccess;
        bool launched = false;
#define ZIPNN_PACK(B_, G_)                                                                                           \
    if (!launched && p.B == B_ && p.g == G_) {                                                                      \
        if (compact)                                                                                                \
            k_compact<B_, G_><<<grid, kBlock, 0, s>>>(d_descs, n_desc, d_chunk_prefix, total_chunks, p, entries,   \
                                                      codes, offsets, totals, nwords);                             \
        else if (xb)   /* the XB instance exists for 2-byte words only */                                        \
            k_pack<B_, G_, B_ == 2><<<grid, kBlock, 0, s>>>(d_descs, n_desc, d_chunk_prefix, total_chunks, p,       \
                                                            entries, codes, offsets, totals, nwords);              \
        else                                                                                                        \
            k_pack<B_, G_, false><<<grid, kBlock, 0, s>>>(d_descs, n_desc, d_chunk_prefix, total_chunks, p, entries,\
                                                          codes, offsets, totals, nwords);                         \
        launched = true;                                                                                            \
    }
        ZIPNN_PACK(1, 2) ZIPNN_PACK(1, 4) ZIPNN_PACK(1, 8)
        ZIPNN_PACK(2, 2) ZIPNN_PACK(2, 4) ZIPNN_PACK(2, 8)
        ZIPNN_PACK(4, 2) ZIPNN_PACK(4, 4) ZIPNN_PACK(4, 8)
#undef ZIPNN_PACK
        if (!launched) return hipErrorInvalidValue;
        return hipGetLastError() == hipSuccess ? hipSuccess : hipErrorLaunchFailure;
    };
    k_place<<<n_desc, kBlock, 0, s>>>(d_descs, p, entries, offsets, totals, nwords);
    if (hipGetLastError() != hipSuccess) return hipErrorLaunchFailure;
    k_arena<<<1, kBlock, 0, s>>>(d_descs, n_desc, p, arena, cap, totals, arena_off);
    if (hipGetLastError() != hipSuccess) return hipErrorLaunchFailure;
    return pack_or_compact(staged);
}

}  // namespace zipnn
