/*
 * ZipNN oracle: a plain, slow, obviously-correct CPU implementation of the
 * byte-grouping + chunked canonical Huffman codec, used ONLY as test
 * infrastructure.  Only the test suite, the smoke check and the benchmark's
 * cpu_baseline leg may load this library; the product path never does.
 *
 * What it computes (ZipNN, arXiv 2411.05239):
 *   - a tensor is a long array of numbers (paper §II-B), cut into fixed-size
 *     chunks that are compressed independently (paper §V-A, "Chunking");
 *   - inside a chunk the words are split into one stream per byte position,
 *     the most significant byte (sign + high exponent bits) first
 *     (paper §III-A "Exponent Extraction", §III-B "Byte Grouping");
 *   - each stream is coded with Huffman only, no LZ stage (paper §III-A
 *     "Huffman only Compression"); a stream holding one value collapses to a
 *     header (paper §III-B), and a stream that does not compress is stored
 *     as is (paper §III-B, §V-B); the decision is per byte-group (§V-A);
 *   - a map with one entry per (chunk, byte-group) lets every chunk decode on
 *     its own (paper §V-A, "Metadata and parallelism");
 *   - optionally the input is first XORed with a base tensor (paper §IV-B).
 * The paper does not fix the Huffman variant or the container bytes.  This
 * file uses: an optimal length-limited code found by package-merge
 * (Larmore & Hirschberg, JACM 1990) with ties broken by (frequency, symbol)
 * and leaves before packages; canonical codes in RFC 1951 §3.2.2 order; code
 * bits most-significant first into an LSB-first bit stream; W interleaved
 * sub-streams of round-robin groups of g symbols; and the 64-byte header /
 * 16-byte map-entry container described in zipnn_oracle.h.
 *
 * Everything here is deliberately simple: bit-by-bit writing and reading,
 * plain loops, no tables beyond the canonical decode counts.
 */
#include "zipnn_oracle.h"

#include <pthread.h>
#include <stdlib.h>
#include <string.h>

/* ---------------------------------------------------------------- helpers */

static int dtype_width(int dtype)
{
    switch (dtype) {
    case ORC_BF16: return 2;
    case ORC_FP16: return 2;
    case ORC_FP32: return 4;
    case ORC_FP8_E4M3: return 1;
    case ORC_U8: return 1;
    default: return 0;
    }
}

static int is_pow2(uint64_t v) { return v != 0 && (v & (v - 1)) == 0; }

static uint64_t align16(uint64_t v) { return (v + 15u) & ~(uint64_t)15u; }

/* Payloads start at multiples of ORC_PAY_ALIGN bytes from the container
 * start, so that a stream never shares a 128-byte memory line with another. */
static uint64_t align_pay(uint64_t v) { return (v + (ORC_PAY_ALIGN - 1)) & ~(uint64_t)(ORC_PAY_ALIGN - 1); }

/* Offset of the payload area: after the header and the map, aligned; a
 * tensor with no chunks is the header alone. */
static uint64_t payload_base_of(uint64_t n_chunks, int B)
{
    return n_chunks ? align_pay(64 + 16 * n_chunks * (uint64_t)B) : 64;
}

static void put_u16(uint8_t* p, uint16_t v) { p[0] = (uint8_t)v; p[1] = (uint8_t)(v >> 8); }
static void put_u32(uint8_t* p, uint32_t v) { for (int i = 0; i < 4; i++) p[i] = (uint8_t)(v >> (8 * i)); }
static void put_u64(uint8_t* p, uint64_t v) { for (int i = 0; i < 8; i++) p[i] = (uint8_t)(v >> (8 * i)); }
static uint16_t get_u16(const uint8_t* p) { return (uint16_t)(p[0] | (p[1] << 8)); }
static uint32_t get_u32(const uint8_t* p)
{
    uint32_t v = 0;
    for (int i = 3; i >= 0; i--) v = (v << 8) | p[i];
    return v;
}
static uint64_t get_u64(const uint8_t* p)
{
    uint64_t v = 0;
    for (int i = 7; i >= 0; i--) v = (v << 8) | p[i];
    return v;
}

int orc_check_params(int B, uint32_t chunk_bytes, uint32_t S, uint32_t g, uint32_t L)
{
    if (B == 0) return ORC_E_INVAL;
    if (!is_pow2(chunk_bytes) || chunk_bytes < ORC_MIN_CHUNK || chunk_bytes > ORC_MAX_CHUNK) return ORC_E_INVAL;
    if (!is_pow2(g) || g < ORC_MIN_G || g > ORC_MAX_G) return ORC_E_INVAL;
    if (!is_pow2(S) || S < g || S > ORC_MAX_S) return ORC_E_INVAL;
    if (L < ORC_MIN_L || L > ORC_MAX_L) return ORC_E_INVAL;
    /* sub-streams per chunk: per stream, and over all B streams */
    if (chunk_bytes / (uint32_t)B / S > ORC_MAX_W || chunk_bytes / S > ORC_MAX_BW) return ORC_E_INVAL;
    return ORC_OK;
}

/* ------------------------------------------------------- byte grouping */

/* Stream k of element j is byte (B-1-k) of the little-endian word, so
 * stream 0 is the most significant byte: sign + exponent bits for BF16,
 * FP16 and FP32 (paper §III-A exponent extraction, §III-B byte grouping). */
void orc_split_stream(const uint8_t* words, uint64_t m, int B, int k, uint8_t* out)
{
    for (uint64_t j = 0; j < m; j++) out[j] = words[j * (uint64_t)B + (uint64_t)(B - 1 - k)];
}

/* Exponent extraction (paper §III-A, "Exponent Extraction"): in a BF16 or
 * FP32 word (sign, 8 exponent bits, fraction from the top) the exponent moves
 * to the top 8 bits and the sign right below it, so that the first byte group
 * holds exactly the exponent.  The fraction bits keep their places.  The
 * m little-endian words of B bytes are rewritten in place; `inverse` undoes
 * it. */
static void exponent_extract(uint8_t* words, uint64_t m, int B, int inverse)
{
    const int nb = 8 * B;
    for (uint64_t i = 0; i < m; i++) {
        uint32_t w = 0;
        for (int b = 0; b < B; b++) w |= (uint32_t)words[i * B + b] << (8 * b);
        const uint32_t frac = w & ((1u << (nb - 9)) - 1);
        uint32_t sign, exp, out;
        if (!inverse) {
            sign = (w >> (nb - 1)) & 1;
            exp = (w >> (nb - 9)) & 0xFF;
            out = (exp << (nb - 8)) | (sign << (nb - 9)) | frac;
        } else {
            exp = (w >> (nb - 8)) & 0xFF;
            sign = (w >> (nb - 9)) & 1;
            out = (sign << (nb - 1)) | (exp << (nb - 9)) | frac;
        }
        for (int b = 0; b < B; b++) words[i * B + b] = (uint8_t)(out >> (8 * b));
    }
}

/* Inverse of orc_split_stream for one stream. */
static void merge_stream(const uint8_t* in, uint64_t m, int B, int k, uint8_t* words)
{
    for (uint64_t j = 0; j < m; j++) words[j * (uint64_t)B + (uint64_t)(B - 1 - k)] = in[j];
}

/* ------------------------------------------------------- package-merge */

typedef struct {
    uint64_t w;   /* weight */
    int leaf;     /* rank of the leaf in the sorted leaf list, or -1 for a package */
} pm_item;

/* Optimal prefix-code lengths with every length <= L (Larmore & Hirschberg
 * package-merge).  Leaves are the symbols with f > 0 in ascending
 * (f, symbol) order.  Starting from the leaf list, L-1 times: pair the
 * current list's items (0+1, 2+3, ...; an odd last item is dropped) into
 * packages whose weight is the sum, then merge the leaves and the packages
 * into the next list by weight, a leaf before a package of equal weight.
 * The first 2n'-2 items of the last list are selected; a selected leaf adds
 * one to its symbol's length and a selected package selects its two
 * children in the list it was made from.  Since the packages of a list are
 * made from consecutive pairs, selecting the first p packages selects the
 * first 2p items of the list below, which is how the expansion is done.
 * Returns the number of coded symbols n', or a negative error. */
int orc_package_merge(const uint64_t f[256], int L, uint8_t len_out[256])
{
    int sym[256];
    int n = 0;
    memset(len_out, 0, 256);
    for (int s = 0; s < 256; s++)
        if (f[s] > 0) sym[n++] = s;
    if (n < 2) return n;               /* zero or one symbol: no code needed */
    if (L < 1 || L > 30 || n > (1 << L)) return ORC_E_INVAL;
    /* insertion sort of the leaves by (f, symbol) -- plain and stable */
    for (int i = 1; i < n; i++) {
        int s = sym[i];
        int j = i - 1;
        while (j >= 0 && (f[sym[j]] > f[s] || (f[sym[j]] == f[s] && sym[j] > s))) {
            sym[j + 1] = sym[j];
            j--;
        }
        sym[j + 1] = s;
    }
    pm_item* lists[32];
    int lens[32];
    int cap = 2 * n;
    for (int d = 0; d < L; d++) {
        lists[d] = (pm_item*)malloc(sizeof(pm_item) * (size_t)cap);
        if (!lists[d]) {
            for (int e = 0; e < d; e++) free(lists[e]);
            return ORC_E_NOMEM;
        }
    }
    /* list 0: the leaves */
    for (int i = 0; i < n; i++) {
        lists[0][i].w = f[sym[i]];
        lists[0][i].leaf = i;
    }
    lens[0] = n;
    for (int d = 1; d < L; d++) {
        const pm_item* prev = lists[d - 1];
        int npk = lens[d - 1] / 2;
        /* merge leaves (i) and packages (p); leaf first on equal weight */
        int i = 0, p = 0, o = 0;
        while (i < n || p < npk) {
            uint64_t pw = 0;
            if (p < npk) pw = prev[2 * p].w + prev[2 * p + 1].w;
            if (i < n && (p >= npk || f[sym[i]] <= pw)) {
                lists[d][o].w = f[sym[i]];
                lists[d][o].leaf = i;
                i++;
            } else {
                lists[d][o].w = pw;
                lists[d][o].leaf = -1;
                p++;
            }
            o++;
        }
        lens[d] = o;
    }
    /* selection, top list first */
    int sel = 2 * n - 2;
    int count[256];
    memset(count, 0, sizeof(count));
    for (int d = L - 1; d >= 0; d--) {
        int npk_sel = 0;
        if (sel > lens[d]) {           /* cannot happen for n <= 2^L */
            for (int e = 0; e < L; e++) free(lists[e]);
            return ORC_E_INVAL;
        }
        for (int t = 0; t < sel; t++) {
            if (lists[d][t].leaf >= 0)
                count[lists[d][t].leaf]++;
            else
                npk_sel++;
        }
        sel = 2 * npk_sel;
    }
    for (int i = 0; i < n; i++) len_out[sym[i]] = (uint8_t)count[i];
    for (int d = 0; d < L; d++) free(lists[d]);
    return n;
}

/* ------------------------------------------------------- canonical codes */

/* RFC 1951 §3.2.2: count the codes of each length, find the first code of
 * each length, then hand out consecutive codes to the symbols of each length
 * in increasing symbol order. */
void orc_canonical_codes(const uint8_t len[256], int L, uint32_t code[256])
{
    uint32_t bl_count[32] = {0};
    uint32_t next_code[32] = {0};
    for (int s = 0; s < 256; s++)
        if (len[s]) bl_count[len[s]]++;
    uint32_t c = 0;
    for (int bits = 1; bits <= L; bits++) {
        c = (c + bl_count[bits - 1]) << 1;
        next_code[bits] = c;
    }
    for (int s = 0; s < 256; s++) {
        code[s] = 0;
        if (len[s]) code[s] = next_code[len[s]]++;
    }
}

/* ------------------------------------------------------- bit I/O */

/* Stream bit i is bit (i mod 8) of byte i/8 (LSB-first); a code goes in most
 * significant code bit first. */
static void put_code(uint8_t* buf, uint64_t* pos, uint32_t code, int len)
{
    for (int b = len - 1; b >= 0; b--) {
        uint32_t bit = (code >> b) & 1u;
        buf[*pos >> 3] |= (uint8_t)(bit << (*pos & 7));
        (*pos)++;
    }
}

/* ------------------------------------------------------- the coding */

/* The bit string of one sub-stream -- the Huffman coding proper (paper
 * §III-A: every byte group is coded with Huffman only).  A stream of m
 * symbols is cut into groups of g consecutive symbols (group q = symbols
 * qg .. min(qg+g, m)-1); with W = ceil(m/S) sub-streams, group q belongs to
 * sub-stream q mod W, so sub-stream w holds the groups w, w+W, w+2W, ... in
 * that order (this spreading of a chunk over W independent sub-streams is
 * the format's own; the paper parallelises over chunks and byte groups only,
 * §V-A).  With flags != NULL (ZG) the groups whose flag is 0 are left out.
 * The bit string is the concatenation of the canonical codes of the symbols,
 * each code most significant bit first; stream bit i is bit i%8 of byte i/8
 * of out (out_bytes bytes, zeroed here).  *nbits receives its length.
 * Returns ORC_OK, ORC_E_INVAL for w >= W or a symbol without a code, or
 * ORC_E_NOSPACE when out is too small. */
int orc_substream_bits(const uint8_t* sym, uint64_t m, uint32_t S, uint32_t g, int L, const uint8_t len[256],
                       const uint8_t* flags, uint64_t w, uint8_t* out, uint64_t out_bytes, uint64_t* nbits)
{
    uint32_t code[256];
    uint64_t W = (m + S - 1) / S;
    uint64_t G = (m + g - 1) / g;
    uint64_t pos = 0;
    if (S == 0 || g == 0 || w >= W) return ORC_E_INVAL;
    orc_canonical_codes(len, L, code);
    memset(out, 0, out_bytes);
    for (uint64_t q = w; q < G; q += W) {
        if (flags && !flags[q]) continue;
        uint64_t end = (q + 1) * g < m ? (q + 1) * g : m;
        for (uint64_t e = q * g; e < end; e++) {
            if (len[sym[e]] == 0) return ORC_E_INVAL;
            if (pos + len[sym[e]] > 8 * out_bytes) return ORC_E_NOSPACE;
            put_code(out, &pos, code[sym[e]], len[sym[e]]);
        }
    }
    *nbits = pos;
    return ORC_OK;
}

/* ------------------------------------------------------- the layout */

/* The word layout of a HUF / ZG payload is the format's choice, not part of
 * the method: the sub-strings are stored so that a decoder that runs 64
 * sub-streams in lock-step (one per lane of a 64-wide wavefront) reads the
 * words it needs next from consecutive addresses.  Sub-streams are taken 64
 * at a time: sub-stream 64j+l is lane l of lane group j.  The layout is
 * defined by the decode events of a lane group:
 *   - the groups of lane l are its steps: the group at step s is
 *     q = 64j + l + s*W; a coded group (every group for HUF, the marked ones
 *     for ZG) gives one event per pair of symbols p = 0, 1, ..., covering
 *     symbols 2p and 2p+1 of the group (the last pair of a short last group
 *     may hold one symbol);
 *   - the events are ordered by (step, pair, lane);
 *   - walking them in that order, a lane whose buffer holds fewer than 2L
 *     bits takes its next 32-bit word (word k = bits 32k .. 32k+31 of its bit
 *     string, zero past the end) before its event, which adds 32 bits to the
 *     buffer; the event's code bits then leave the buffer.
 * The words of a lane group are stored in the order they are taken, and the
 * lane groups one after another.  2L bits cover the two codes of a pair, so a
 * decoder always holds the bits it is about to read; near the end a lane may
 * take one word that lies wholly past its last code bit (all zero). */

typedef struct {
    uint64_t step;
    uint32_t pair;
    uint32_t lane;
    uint32_t bits;   /* code bits of the pair's symbols (0 when not known yet) */
} lg_event;

static int event_order(const void* a, const void* b)
{
    const lg_event* x = (const lg_event*)a;
    const lg_event* y = (const lg_event*)b;
    if (x->step != y->step) return x->step < y->step ? -1 : 1;
    if (x->pair != y->pair) return x->pair < y->pair ? -1 : 1;
    if (x->lane != y->lane) return x->lane < y->lane ? -1 : 1;
    return 0;
}

/* The events of lane group j, sorted.  flags: NULL (every group coded) or
 * one byte per group.  With len != NULL each event carries the length of its
 * codes (sym is then read); else 0.  *n_ev receives their number; NULL on an
 * allocation failure. */
static lg_event* lane_group_events(const uint8_t* sym, const uint8_t* len, uint64_t m, uint32_t S, uint32_t g,
                                   const uint8_t* flags, uint64_t j, uint64_t* n_ev)
{
    uint64_t W = (m + S - 1) / S;
    uint64_t G = (m + g - 1) / g;
    uint64_t lanes = W - ORC_LANES * j < ORC_LANES ? W - ORC_LANES * j : ORC_LANES;
    uint64_t steps = (G + W - 1) / W;
    uint64_t cap = lanes * steps * ((g + 1) / 2) + 1;
    lg_event* ev = (lg_event*)malloc(sizeof(lg_event) * cap);
    uint64_t n = 0;
    if (!ev) return NULL;
    for (uint64_t l = 0; l < lanes; l++) {
        for (uint64_t s = 0; s < steps; s++) {
            uint64_t q = ORC_LANES * j + l + s * W;
            if (q >= G || (flags && !flags[q])) continue;
            uint64_t cnt = (q + 1) * g <= m ? g : m - q * g;
            for (uint64_t p = 0; 2 * p < cnt; p++) {
                uint32_t bits = 0;
                if (len) {
                    bits = len[sym[q * g + 2 * p]];
                    if (2 * p + 1 < cnt) bits += len[sym[q * g + 2 * p + 1]];
                }
                ev[n].step = s;
                ev[n].pair = (uint32_t)p;
                ev[n].lane = (uint32_t)l;
                ev[n].bits = bits;
                n++;
            }
        }
    }
    qsort(ev, n, sizeof(lg_event), event_order);
    *n_ev = n;
    return ev;
}

/* Lay out one lane group: the lanes' bit strings (lane l at bits +
 * l*lane_bytes, each long enough for the word taken past its end) become the
 * word sequence defined above, written to words; returns the word count. */
static uint64_t interleave(const lg_event* ev, uint64_t n_ev, const uint8_t* bits, uint64_t lane_bytes, int L,
                           uint8_t* words)
{
    int64_t buffered[ORC_LANES];
    uint64_t taken[ORC_LANES];
    uint64_t n = 0;
    memset(buffered, 0, sizeof(buffered));
    memset(taken, 0, sizeof(taken));
    for (uint64_t i = 0; i < n_ev; i++) {
        uint32_t l = ev[i].lane;
        if (buffered[l] < 2 * L) {
            put_u32(words + 4 * n, get_u32(bits + l * lane_bytes + 4 * taken[l]));
            n++;
            taken[l]++;
            buffered[l] += 32;
        }
        buffered[l] -= ev[i].bits;
    }
    return n;
}

/* ------------------------------------------------------- per-stream coding */

typedef struct {
    int mode;           /* ORC_MODE_* */
    uint8_t rle;        /* value of an RLE stream */
    uint64_t bytes;     /* payload bytes */
    uint8_t* payload;   /* malloc'd (NULL for RLE) */
} stream_out;

/* Bytes of a HUF payload before its word streams: the nibble table, one u32
 * word count per lane group, zero padding to 16. */
static uint64_t huf_head_bytes(uint64_t W)
{
    return align16(128 + 4 * ((W + ORC_LANES - 1) / ORC_LANES));
}

/* Bytes of the group bitmap of a ZG payload: one bit per group of g symbols,
 * zero padded to 16. */
static uint64_t zg_bitmap_bytes(uint64_t m, uint32_t g)
{
    return align16(((m + g - 1) / g + 7) / 8);
}

/* The Huffman payload of m symbols with the given code lengths: the 4-bit
 * length table, the word count of each lane group, (ZG: the group bitmap,)
 * then each lane group's sub-stream bit strings laid out as described above.
 * flags == NULL: HUF, every group coded; else ZG, the groups q with flags[q]
 * set are coded and marked in the bitmap. */
static int huf_payload(const uint8_t* sym, uint64_t m, uint32_t S, uint32_t g, int L, const uint8_t len[256],
                       const uint8_t* flags, stream_out* out)
{
    uint64_t W = (m + S - 1) / S;
    uint64_t NG = (W + ORC_LANES - 1) / ORC_LANES;
    uint64_t H = huf_head_bytes(W);
    uint64_t G = (m + g - 1) / g;
    uint64_t BM = flags ? zg_bitmap_bytes(m, g) : 0;
    uint64_t steps = (G + W - 1) / W;                          /* groups of the longest sub-stream */
    uint64_t nmax = steps * g;                                 /* symbols of the longest sub-stream */
    uint64_t lane_bytes = ((nmax * (uint64_t)L + 31) / 32 + 1) * 4;   /* its words + the one past the end */
    uint64_t max_words = W * (lane_bytes / 4);
    uint8_t* p = (uint8_t*)calloc(H + BM + 4 * max_words, 1);
    uint8_t* bits = (uint8_t*)malloc(ORC_LANES * lane_bytes);
    if (!p || !bits) {
        free(p);
        free(bits);
        return ORC_E_NOMEM;
    }
    for (int i = 0; i < 128; i++) p[i] = (uint8_t)(len[2 * i] | (len[2 * i + 1] << 4));
    if (flags)
        for (uint64_t q = 0; q < G; q++)
            if (flags[q]) p[H + q / 8] |= (uint8_t)(1u << (q % 8));
    uint8_t* words = p + H + BM;
    uint64_t wpos = 0;
    int rc = ORC_OK;
    for (uint64_t j = 0; j < NG && rc == ORC_OK; j++) {
        uint64_t lanes = W - ORC_LANES * j < ORC_LANES ? W - ORC_LANES * j : ORC_LANES;
        uint64_t nbits, n_ev;
        for (uint64_t l = 0; l < lanes && rc == ORC_OK; l++)
            rc = orc_substream_bits(sym, m, S, g, L, len, flags, ORC_LANES * j + l, bits + l * lane_bytes, lane_bytes,
                                    &nbits);
        if (rc != ORC_OK) break;
        lg_event* ev = lane_group_events(sym, len, m, S, g, flags, j, &n_ev);
        if (!ev) {
            rc = ORC_E_NOMEM;
            break;
        }
        uint64_t nw = interleave(ev, n_ev, bits, lane_bytes, L, words + 4 * wpos);
        free(ev);
        put_u32(p + 128 + 4 * j, (uint32_t)nw);
        wpos += nw;
    }
    free(bits);
    if (rc != ORC_OK) {
        free(p);
        return rc;
    }
    out->mode = flags ? ORC_MODE_ZG : ORC_MODE_HUF;
    out->bytes = H + BM + 4 * wpos;
    out->payload = p;
    return ORC_OK;
}

/* Encode one byte-group (stream) of one chunk: m symbols.  The method
 * decision is made per byte-group (paper §V-A):
 *   - RAW when the policy says so;
 *   - RLE when the stream holds a single value (paper §III-B: a zero stream
 *     is replaced by a header -- generalised to any single value);
 *   - HUF: Huffman coding of every symbol (paper §III-A);
 *   - ZG: the stream's most frequent value z (smallest on ties) fills every
 *     group of g symbols made of z alone; a bitmap marks the other groups,
 *     whose symbols are Huffman coded.  This is the zero-aware coding of
 *     deltas (paper §IV-B: mostly unchanged bytes, whose XOR is zero) done
 *     without an LZ stage.
 * Under AUTO the smallest of RAW, HUF and (when z fills at least half of the
 * symbols) ZG is kept, ties going to RAW, then HUF; incompressible groups
 * stay raw (paper §III-B, §V-B).  Policy HUF forces HUF; policy ZG forces
 * ZG when the coded groups hold two distinct values at least, else HUF. */
static int encode_stream(const uint8_t* sym, uint64_t m, uint32_t S, uint32_t g, int L, int policy,
                         stream_out* out)
{
    memset(out, 0, sizeof(*out));
    if (policy == ORC_POLICY_RAW) goto raw;
    uint64_t f[256];
    memset(f, 0, sizeof(f));
    for (uint64_t j = 0; j < m; j++) f[sym[j]]++;
    int distinct = 0;
    int only = 0, z = 0;
    for (int s = 0; s < 256; s++) {
        if (f[s]) {
            distinct++;
            only = s;
        }
        if (f[s] > f[z]) z = s;
    }
    if (distinct == 1) {
        out->mode = ORC_MODE_RLE;
        out->rle = (uint8_t)only;
        out->bytes = 0;
        return ORC_OK;
    }
    stream_out huf, zg;
    memset(&huf, 0, sizeof(huf));
    memset(&zg, 0, sizeof(zg));
    int have_huf = 0, have_zg = 0;
    if (policy != ORC_POLICY_ZG) {
        uint8_t len[256];
        int rc = orc_package_merge(f, L, len);
        if (rc < 0) return rc;
        rc = huf_payload(sym, m, S, g, L, len, NULL, &huf);
        if (rc != ORC_OK) return rc;
        have_huf = 1;
    }
    if (policy == ORC_POLICY_ZG || (policy == ORC_POLICY_AUTO && 2 * f[z] >= m)) {
        uint64_t G = (m + g - 1) / g;
        uint8_t* flags = (uint8_t*)calloc(G ? G : 1, 1);
        uint64_t f2[256];
        memset(f2, 0, sizeof(f2));
        if (!flags) return ORC_E_NOMEM;
        for (uint64_t q = 0; q < G; q++) {
            uint64_t end = (q + 1) * g < m ? (q + 1) * g : m;
            for (uint64_t e = q * g; e < end; e++)
                if (sym[e] != z) flags[q] = 1;
            if (flags[q])
                for (uint64_t e = q * g; e < end; e++) f2[sym[e]]++;
        }
        int d2 = 0;
        for (int s = 0; s < 256; s++) d2 += f2[s] != 0;
        if (d2 >= 2) {
            uint8_t len2[256];
            int rc = orc_package_merge(f2, L, len2);
            if (rc >= 0) rc = huf_payload(sym, m, S, g, L, len2, flags, &zg);
            if (rc < 0) {
                free(flags);
                free(huf.payload);
                return rc;
            }
            zg.rle = (uint8_t)z;
            have_zg = 1;
        }
        free(flags);
        if (!have_zg && !have_huf) {   /* forced ZG without two coded values: HUF */
            uint8_t len[256];
            int rc = orc_package_merge(f, L, len);
            if (rc >= 0) rc = huf_payload(sym, m, S, g, L, len, NULL, &huf);
            if (rc < 0) return rc;
            have_huf = 1;
        }
    }
    if (policy == ORC_POLICY_AUTO) {
        uint64_t best = m;
        int pick = 0;   /* 0 raw, 1 huf, 2 zg */
        if (have_huf && huf.bytes < best) {
            best = huf.bytes;
            pick = 1;
        }
        if (have_zg && zg.bytes < best) pick = 2;
        if (pick != 1) free(huf.payload);
        if (pick != 2) free(zg.payload);
        if (pick == 0) goto raw;
        *out = pick == 1 ? huf : zg;
        return ORC_OK;
    }
    if (have_zg) {
        free(huf.payload);
        *out = zg;
    } else {
        *out = huf;
    }
    return ORC_OK;

raw:
    out->mode = ORC_MODE_RAW;
    out->bytes = m;
    out->payload = (uint8_t*)malloc(m ? m : 1);
    if (!out->payload) return ORC_E_NOMEM;
    memcpy(out->payload, sym, m);
    return ORC_OK;
}

/* Decode a Huffman (zg = 0) or ZG (zg = 1, fill value z) payload of m
 * symbols.  The groups a ZG bitmap leaves unmarked are filled with z.  Each
 * lane group is read back by walking its sorted decode events (see "the
 * layout" above): before an event, a lane holding fewer than 2L unread bits
 * takes the next word of the lane group's sequence; then the event's one or
 * two symbols are read from the lane's bits one bit at a time, each code
 * being recognised by canonical decoding.  Returns ORC_OK or ORC_E_CORRUPT. */
static int decode_huf(const uint8_t* p, uint64_t bytes, uint64_t m, uint32_t S, uint32_t g, int L, int zg,
                      uint8_t z, uint8_t* sym)
{
    uint64_t W = (m + S - 1) / S;
    uint64_t NG = (W + ORC_LANES - 1) / ORC_LANES;
    uint64_t H = huf_head_bytes(W);
    uint64_t G = (m + g - 1) / g;
    uint64_t BM = zg ? zg_bitmap_bytes(m, g) : 0;
    if (bytes < H + BM) return ORC_E_CORRUPT;
    uint8_t len[256];
    for (int i = 0; i < 128; i++) {
        len[2 * i] = p[i] & 15;
        len[2 * i + 1] = p[i] >> 4;
    }
    /* the table must be a complete prefix code: at least two symbols, no
     * length above L, Kraft sum exactly one */
    int n_coded = 0;
    uint64_t kraft = 0;
    for (int s = 0; s < 256; s++) {
        if (!len[s]) continue;
        if (len[s] > L) return ORC_E_CORRUPT;
        n_coded++;
        kraft += (uint64_t)1 << (L - len[s]);
    }
    if (n_coded < 2 || kraft != ((uint64_t)1 << L)) return ORC_E_CORRUPT;
    for (uint64_t i = 128 + 4 * NG; i < H; i++)
        if (p[i] != 0) return ORC_E_CORRUPT;
    /* bitmap: no bit past the last group */
    for (uint64_t q = G; q < 8 * BM; q++)
        if ((p[H + q / 8] >> (q % 8)) & 1) return ORC_E_CORRUPT;
    uint64_t total = 0;
    for (uint64_t j = 0; j < NG; j++) total += get_u32(p + 128 + 4 * j);
    if (bytes != H + BM + 4 * total) return ORC_E_CORRUPT;
    const uint8_t* words = p + H + BM;

    /* ZG: the coded groups are the marked ones; the others hold z */
    uint8_t* flags = NULL;
    if (zg) {
        flags = (uint8_t*)malloc(G ? G : 1);
        if (!flags) return ORC_E_NOMEM;
        for (uint64_t q = 0; q < G; q++) {
            flags[q] = (uint8_t)((p[H + q / 8] >> (q % 8)) & 1);
            if (!flags[q]) {
                uint64_t end = (q + 1) * g < m ? (q + 1) * g : m;
                memset(sym + q * g, z, end - q * g);
            }
        }
    }

    /* canonical decoding tables: symbols sorted by (length, symbol) and the
     * count of codes of each length */
    int count[32] = {0};
    int sorted[256];
    int ns = 0;
    for (int l = 1; l <= L; l++)
        for (int s = 0; s < 256; s++)
            if (len[s] == l) {
                sorted[ns++] = s;
                count[l]++;
            }
    uint64_t steps = (G + W - 1) / W;
    uint64_t nmax = steps * g;
    uint64_t max_take = (nmax * (uint64_t)L + 2 * L) / 32 + 2;   /* words a lane can take */
    uint32_t* got = (uint32_t*)malloc(sizeof(uint32_t) * ORC_LANES * max_take);
    if (!got) {
        free(flags);
        return ORC_E_NOMEM;
    }
    int rc = ORC_OK;
    uint64_t wpos = 0;
    for (uint64_t j = 0; j < NG && rc == ORC_OK; j++) {
        uint64_t taken[ORC_LANES], bitpos[ORC_LANES];
        int64_t buffered[ORC_LANES];
        memset(taken, 0, sizeof(taken));
        memset(bitpos, 0, sizeof(bitpos));
        memset(buffered, 0, sizeof(buffered));
        uint64_t end = wpos + get_u32(p + 128 + 4 * j);
        uint64_t n_ev;
        lg_event* ev = lane_group_events(NULL, NULL, m, S, g, flags, j, &n_ev);
        if (!ev) {
            rc = ORC_E_NOMEM;
            break;
        }
        for (uint64_t i = 0; i < n_ev && rc == ORC_OK; i++) {
            uint32_t l = ev[i].lane;
            uint64_t q = ORC_LANES * j + l + ev[i].step * W;
            uint64_t cnt = (q + 1) * g <= m ? g : m - q * g;
            if (buffered[l] < 2 * L) {
                if (wpos >= end || taken[l] >= max_take) {
                    rc = ORC_E_CORRUPT;
                    break;
                }
                got[l * max_take + taken[l]++] = get_u32(words + 4 * wpos++);
                buffered[l] += 32;
            }
            for (uint64_t t = 2 * (uint64_t)ev[i].pair; t < 2 * (uint64_t)ev[i].pair + 2 && t < cnt; t++) {
                /* read code bits one at a time; after b bits, the code value
                 * minus the first code of length b is the index among the
                 * symbols of length b if below their count */
                int codev = 0, first = 0, index = 0, found = -1;
                for (int b = 1; b <= L; b++) {
                    if (bitpos[l] >= 32 * taken[l]) break;
                    uint32_t wd = got[l * max_take + bitpos[l] / 32];
                    codev |= (int)((wd >> (bitpos[l] % 32)) & 1u);
                    bitpos[l]++;
                    buffered[l]--;
                    if (codev - first < count[b]) {
                        found = sorted[index + codev - first];
                        break;
                    }
                    index += count[b];
                    first += count[b];
                    first <<= 1;
                    codev <<= 1;
                }
                if (found < 0) {
                    rc = ORC_E_CORRUPT;
                    break;
                }
                sym[q * g + t] = (uint8_t)found;
            }
        }
        free(ev);
        if (rc == ORC_OK && wpos != end) rc = ORC_E_CORRUPT;   /* every word taken exactly */
    }
    free(got);
    free(flags);
    return rc;
}

/* ------------------------------------------------------- chunk workers */

typedef struct {
    const uint8_t* src;
    const uint8_t* base;
    uint64_t n;
    int B;
    uint32_t E;           /* elements per chunk */
    uint32_t S, g;
    int L;
    const uint8_t* policy;
    uint32_t skip;        /* probe interval K (0: every chunk is analysed) */
    int exp;              /* exponent extraction before the split */
    int phase;            /* 0: probe chunks, 1: the others */
    stream_out* outs;     /* n_chunks * B */
    uint32_t n_chunks;
    uint32_t next;        /* next chunk to take */
    pthread_mutex_t mu;
    int rc;
} enc_job;

static int encode_chunk(enc_job* J, uint32_t c)
{
    uint64_t e0 = (uint64_t)c * J->E;
    uint64_t m = J->n - e0 < J->E ? J->n - e0 : J->E;
    uint8_t* words = (uint8_t*)malloc(m * (uint64_t)J->B);
    uint8_t* s = (uint8_t*)malloc(m);
    if (!words || !s) {
        free(words);
        free(s);
        return ORC_E_NOMEM;
    }
    /* XOR delta against the base (paper §IV-B), bytewise */
    for (uint64_t i = 0; i < m * (uint64_t)J->B; i++) {
        uint8_t x = J->src[e0 * J->B + i];
        words[i] = J->base ? (uint8_t)(x ^ J->base[e0 * J->B + i]) : x;
    }
    if (J->exp) exponent_extract(words, m, J->B, 0);
    int rc = ORC_OK;
    for (int k = 0; k < J->B && rc == ORC_OK; k++) {
        /* compressibility probing (paper §III-B, "Identifying compressibility"):
         * under AUTO, a chunk that is not a probe chunk is stored raw without
         * analysis when its run's probe chunk came out raw */
        int policy = J->policy[k];
        uint32_t run = J->skip + 1;
        if (policy == ORC_POLICY_AUTO && c % run != 0 &&
            J->outs[(uint64_t)(c - c % run) * J->B + k].mode == ORC_MODE_RAW)
            policy = ORC_POLICY_RAW;
        orc_split_stream(words, m, J->B, k, s);
        rc = encode_stream(s, m, J->S, J->g, J->L, policy, &J->outs[(uint64_t)c * J->B + k]);
    }
    free(words);
    free(s);
    return rc;
}

static void* enc_worker(void* arg)
{
    enc_job* J = (enc_job*)arg;
    for (;;) {
        pthread_mutex_lock(&J->mu);
        uint32_t c = J->next++;
        int stop = J->rc != ORC_OK;
        pthread_mutex_unlock(&J->mu);
        if (stop || c >= J->n_chunks) break;
        if ((c % (J->skip + 1) == 0) != (J->phase == 0)) continue;   /* the other phase's chunk */
        int rc = encode_chunk(J, c);
        if (rc != ORC_OK) {
            pthread_mutex_lock(&J->mu);
            if (J->rc == ORC_OK) J->rc = rc;
            pthread_mutex_unlock(&J->mu);
        }
    }
    return NULL;
}

static void run_threads(void* (*fn)(void*), void* job, int nthreads)
{
    if (nthreads <= 1) {
        fn(job);
        return;
    }
    pthread_t* th = (pthread_t*)malloc(sizeof(pthread_t) * (size_t)nthreads);
    int started = 0;
    for (int t = 0; t < nthreads; t++)
        if (pthread_create(&th[t], NULL, fn, job) == 0) started++;
        else break;
    if (started == 0) fn(job);
    for (int t = 0; t < started; t++) pthread_join(th[t], NULL);
    free(th);
}

/* ------------------------------------------------------- public API */

uint64_t orc_compress_bound(int dtype, uint64_t n, uint32_t chunk_bytes, uint32_t S)
{
    int B = dtype_width(dtype);
    if (!B || !is_pow2(chunk_bytes) || S == 0) return 0;
    uint64_t E = chunk_bytes / (uint64_t)B;
    uint64_t nc = (n + E - 1) / E;
    uint64_t W = (E + S - 1) / S;
    /* per stream: a raw copy, or (HUF or ZG forced) the head, a ZG bitmap of
     * at most one bit per two symbols, at most L <= 11 bits per symbol and
     * two extra words per sub-stream; plus alignment */
    uint64_t huf = 128 + 4 * (W / ORC_LANES + 1) + 16 + (E / 16 + 16) + (E * 11 + 7) / 8 + 8 * W + 8;
    uint64_t per_stream = (huf > E ? huf : E) + ORC_PAY_ALIGN;
    return 64 + ORC_PAY_ALIGN + nc * (uint64_t)B * (16 + per_stream);
}

int orc_compress(const void* src_v, int dtype, uint64_t n, const void* base_v, uint32_t chunk_bytes,
                 uint32_t S, uint32_t g, uint32_t L, const uint8_t* policy_in, uint32_t skip, int exp,
                 void* dst_v, uint64_t dst_cap, uint64_t* dst_len, int nthreads)
{
    const uint8_t* src = (const uint8_t*)src_v;
    const uint8_t* base = (const uint8_t*)base_v;
    uint8_t* dst = (uint8_t*)dst_v;
    int B = dtype_width(dtype);
    if (!B || (!src && n) || !dst || !dst_len) return ORC_E_INVAL;
    int rc = orc_check_params(B, chunk_bytes, S, g, L);
    if (rc) return rc;
    uint8_t policy[4] = {0, 0, 0, 0};
    for (int k = 0; k < B; k++) {
        policy[k] = policy_in ? policy_in[k] : ORC_POLICY_AUTO;
        if (policy[k] > ORC_POLICY_ZG) return ORC_E_INVAL;
    }
    if (skip > 255) return ORC_E_INVAL;
    if (exp && dtype != ORC_BF16 && dtype != ORC_FP32) return ORC_E_INVAL;
    uint32_t E = chunk_bytes / (uint32_t)B;
    uint64_t nc64 = (n + E - 1) / E;
    if (nc64 > 0xFFFFFFFFu) return ORC_E_INVAL;
    uint32_t n_chunks = (uint32_t)nc64;

    enc_job J;
    memset(&J, 0, sizeof(J));
    J.src = src;
    J.base = base;
    J.n = n;
    J.B = B;
    J.E = E;
    J.S = S;
    J.g = g;
    J.L = (int)L;
    J.policy = policy;
    J.skip = skip;
    J.exp = exp != 0;
    J.n_chunks = n_chunks;
    J.outs = (stream_out*)calloc((size_t)n_chunks * B + 1, sizeof(stream_out));
    if (!J.outs) return ORC_E_NOMEM;
    pthread_mutex_init(&J.mu, NULL);
    /* probe chunks first, then the chunks that follow them */
    for (J.phase = 0; J.phase < 2 && J.rc == ORC_OK; J.phase++) {
        J.next = 0;
        run_threads(enc_worker, &J, nthreads);
    }
    pthread_mutex_destroy(&J.mu);
    rc = J.rc;

    /* placement: chunk-major order, every payload aligned */
    uint64_t payload_base = payload_base_of(n_chunks, B);
    uint64_t cur = 0;
    if (rc == ORC_OK) {
        for (uint64_t e = 0; e < (uint64_t)n_chunks * B; e++)
            if (J.outs[e].bytes) cur = align_pay(cur + J.outs[e].bytes);
        if (payload_base + cur > dst_cap) rc = ORC_E_NOSPACE;
    }
    if (rc == ORC_OK) {
        uint64_t total = payload_base + cur;
        memset(dst, 0, total);
        memcpy(dst, "ZNN1", 4);
        put_u16(dst + 4, 1);
        dst[6] = (uint8_t)dtype;
        dst[7] = (uint8_t)B;
        put_u64(dst + 8, n);
        put_u32(dst + 16, chunk_bytes);
        put_u16(dst + 20, (uint16_t)S);
        dst[22] = (uint8_t)g;
        dst[23] = (uint8_t)L;
        uint32_t fl = (base ? ORC_FLAG_DELTA : 0) | (exp ? ORC_FLAG_EXP : 0);
        for (uint64_t e = 0; e < (uint64_t)n_chunks * B; e++)
            if (J.outs[e].mode == ORC_MODE_ZG) fl |= ORC_FLAG_ZG;
        put_u32(dst + 24, fl);
        put_u32(dst + 28, n_chunks);
        put_u64(dst + 32, total);
        for (int k = 0; k < 4; k++) dst[40 + k] = policy[k];
        dst[44] = (uint8_t)skip;
        cur = 0;
        for (uint64_t e = 0; e < (uint64_t)n_chunks * B; e++) {
            uint8_t* ent = dst + 64 + 16 * e;
            stream_out* o = &J.outs[e];
            put_u64(ent, cur);
            put_u32(ent + 8, (uint32_t)o->bytes);
            ent[12] = (uint8_t)o->mode;
            ent[13] = o->mode == ORC_MODE_RLE || o->mode == ORC_MODE_ZG ? o->rle : 0;
            if (o->bytes) {
                memcpy(dst + payload_base + cur, o->payload, o->bytes);
                cur = align_pay(cur + o->bytes);
            }
        }
        *dst_len = total;
    }
    for (uint64_t e = 0; e < (uint64_t)n_chunks * B; e++) free(J.outs[e].payload);
    free(J.outs);
    return rc;
}

int orc_parse_header(const void* src_v, uint64_t src_len, orc_header* h)
{
    const uint8_t* src = (const uint8_t*)src_v;
    if (!src || src_len < 64) return ORC_E_FORMAT;
    if (memcmp(src, "ZNN1", 4) != 0 || get_u16(src + 4) != 1) return ORC_E_FORMAT;
    h->dtype = src[6];
    h->B = src[7];
    h->n = get_u64(src + 8);
    h->chunk_bytes = get_u32(src + 16);
    h->S = get_u16(src + 20);
    h->g = src[22];
    h->L = src[23];
    h->flags = get_u32(src + 24);
    h->n_chunks = get_u32(src + 28);
    h->total = get_u64(src + 32);
    for (int k = 0; k < 4; k++) h->policy[k] = src[40 + k];
    h->skip = src[44];
    if (dtype_width(h->dtype) == 0 || dtype_width(h->dtype) != h->B) return ORC_E_FORMAT;
    if (orc_check_params(h->B, h->chunk_bytes, h->S, h->g, h->L) != ORC_OK) return ORC_E_FORMAT;
    if (h->flags & ~(uint32_t)(ORC_FLAG_DELTA | ORC_FLAG_ZG | ORC_FLAG_EXP)) return ORC_E_FORMAT;
    if ((h->flags & ORC_FLAG_EXP) && h->dtype != ORC_BF16 && h->dtype != ORC_FP32) return ORC_E_FORMAT;
    for (int i = 45; i < 64; i++)
        if (src[i]) return ORC_E_FORMAT;
    uint64_t E = h->chunk_bytes / h->B;
    if ((h->n + E - 1) / E != h->n_chunks) return ORC_E_FORMAT;
    uint64_t payload_base = payload_base_of(h->n_chunks, h->B);
    if (h->total < payload_base || h->total > src_len) return ORC_E_FORMAT;
    return ORC_OK;
}

typedef struct {
    const uint8_t* src;
    const uint8_t* base;
    uint8_t* dst;
    orc_header h;
    uint32_t next;
    pthread_mutex_t mu;
    int rc;
} dec_job;

static int decode_chunk(dec_job* J, uint32_t c)
{
    const orc_header* h = &J->h;
    uint64_t E = h->chunk_bytes / h->B;
    uint64_t e0 = (uint64_t)c * E;
    uint64_t m = h->n - e0 < E ? h->n - e0 : E;
    uint64_t payload_base = payload_base_of(h->n_chunks, h->B);
    uint8_t* s = (uint8_t*)malloc(m);
    uint8_t* words = (uint8_t*)malloc(m * h->B);
    if (!s || !words) {
        free(s);
        free(words);
        return ORC_E_NOMEM;
    }
    int rc = ORC_OK;
    for (int k = 0; k < h->B && rc == ORC_OK; k++) {
        const uint8_t* ent = J->src + 64 + 16 * ((uint64_t)c * h->B + k);
        uint64_t off = get_u64(ent);
        uint64_t bytes = get_u32(ent + 8);
        int mode = ent[12];
        const uint8_t* p = J->src + payload_base + off;
        if (mode == ORC_MODE_RAW) {
            memcpy(s, p, m);
        } else if (mode == ORC_MODE_RLE) {
            memset(s, ent[13], m);
        } else {
            rc = decode_huf(p, bytes, m, h->S, h->g, h->L, mode == ORC_MODE_ZG, ent[13], s);
        }
        if (rc == ORC_OK) merge_stream(s, m, h->B, k, words);
    }
    if (rc == ORC_OK) {
        if (h->flags & ORC_FLAG_EXP) exponent_extract(words, m, h->B, 1);
        for (uint64_t i = 0; i < m * h->B; i++) {
            uint8_t y = words[i];
            J->dst[e0 * h->B + i] = J->base ? (uint8_t)(y ^ J->base[e0 * h->B + i]) : y;
        }
    }
    free(s);
    free(words);
    return rc;
}

static void* dec_worker(void* arg)
{
    dec_job* J = (dec_job*)arg;
    for (;;) {
        pthread_mutex_lock(&J->mu);
        uint32_t c = J->next++;
        int stop = J->rc != ORC_OK;
        pthread_mutex_unlock(&J->mu);
        if (stop || c >= J->h.n_chunks) break;
        int rc = decode_chunk(J, c);
        if (rc != ORC_OK) {
            pthread_mutex_lock(&J->mu);
            if (J->rc == ORC_OK) J->rc = rc;
            pthread_mutex_unlock(&J->mu);
        }
    }
    return NULL;
}

/* Check every map entry before touching a payload: modes, sizes and the
 * exact chunk-major, aligned placement. */
static int check_map(const uint8_t* src, const orc_header* h)
{
    uint64_t E = h->chunk_bytes / h->B;
    uint64_t payload_base = payload_base_of(h->n_chunks, h->B);
    uint64_t cur = 0;
    for (uint64_t c = 0; c < h->n_chunks; c++) {
        uint64_t m = h->n - c * E < E ? h->n - c * E : E;
        uint64_t W = (m + h->S - 1) / h->S;
        for (int k = 0; k < h->B; k++) {
            const uint8_t* ent = src + 64 + 16 * (c * h->B + k);
            uint64_t off = get_u64(ent);
            uint64_t bytes = get_u32(ent + 8);
            int mode = ent[12];
            if (ent[14] || ent[15]) return ORC_E_CORRUPT;
            if (off != cur) return ORC_E_CORRUPT;
            if (mode == ORC_MODE_RAW) {
                if (bytes != m || ent[13]) return ORC_E_CORRUPT;
            } else if (mode == ORC_MODE_RLE) {
                if (bytes != 0) return ORC_E_CORRUPT;
            } else if (mode == ORC_MODE_HUF) {
                if (bytes < huf_head_bytes(W) || ent[13]) return ORC_E_CORRUPT;
            } else if (mode == ORC_MODE_ZG) {
                /* a ZG entry needs the header's ZG flag */
                if (!(h->flags & ORC_FLAG_ZG) || bytes < huf_head_bytes(W) + zg_bitmap_bytes(m, h->g))
                    return ORC_E_CORRUPT;
            } else {
                return ORC_E_CORRUPT;
            }
            if (payload_base + off + bytes > h->total) return ORC_E_CORRUPT;
            if (bytes) cur = align_pay(cur + bytes);
        }
    }
    if (payload_base + cur != h->total) return ORC_E_CORRUPT;
    return ORC_OK;
}

int orc_decompress(const void* src_v, uint64_t src_len, const void* base_v, void* dst_v, uint64_t dst_cap,
                   int nthreads)
{
    const uint8_t* src = (const uint8_t*)src_v;
    orc_header h;
    int rc = orc_parse_header(src, src_len, &h);
    if (rc) return rc;
    if ((h.flags & ORC_FLAG_DELTA) && !base_v) return ORC_E_INVAL;
    if (!(h.flags & ORC_FLAG_DELTA) && base_v) return ORC_E_INVAL;
    if (h.n * h.B > dst_cap) return ORC_E_NOSPACE;
    if (h.n && !dst_v) return ORC_E_INVAL;
    rc = check_map(src, &h);
    if (rc) return rc;
    dec_job J;
    memset(&J, 0, sizeof(J));
    J.src = src;
    J.base = (const uint8_t*)base_v;
    J.dst = (uint8_t*)dst_v;
    J.h = h;
    pthread_mutex_init(&J.mu, NULL);
    run_threads(dec_worker, &J, nthreads);
    pthread_mutex_destroy(&J.mu);
    return J.rc;
}

/* Payload of one (chunk, stream) entry, for per-chunk parity sampling. */
int orc_entry(const void* src_v, uint64_t src_len, uint32_t chunk, int k, uint64_t* off_abs, uint64_t* bytes,
              int* mode, int* rle)
{
    const uint8_t* src = (const uint8_t*)src_v;
    orc_header h;
    int rc = orc_parse_header(src, src_len, &h);
    if (rc) return rc;
    if (chunk >= h.n_chunks || k < 0 || k >= h.B) return ORC_E_INVAL;
    const uint8_t* ent = src + 64 + 16 * ((uint64_t)chunk * h.B + k);
    *off_abs = payload_base_of(h.n_chunks, h.B) + get_u64(ent);
    *bytes = get_u32(ent + 8);
    *mode = ent[12];
    *rle = ent[13];
    return ORC_OK;
}
