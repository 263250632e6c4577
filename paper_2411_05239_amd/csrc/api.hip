// Host runtime behind include/zipnn.h: contexts, argument checks, scratch
// management, kernel launches and host-side container inspection.
#include <mutex>
#include <new>
#include <string.h>

#include "zipnn_internal.h"

using namespace zipnn;

struct zipnn_ctx_s {
    int device = 0;
    int dec_grid = 1024;
    int* d_status = nullptr;      // sticky device-side status
    int* h_status = nullptr;      // pinned
    uint64_t* h_total = nullptr;  // pinned, encode sizes
    size_t h_total_cap = 0;
    void* d_scratch = nullptr;    // encode scratch (grown on demand)
    size_t scratch_cap = 0;
    std::mutex mu;                // serialises users of the scratch
};

namespace {

struct DeviceGuard {
    int prev = -1;
    explicit DeviceGuard(int dev)
    {
        if (hipGetDevice(&prev) != hipSuccess) prev = -1;
        if (prev != dev) (void)hipSetDevice(dev);
    }
    ~DeviceGuard()
    {
        if (prev >= 0) (void)hipSetDevice(prev);
    }
};

bool aligned16(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 15u) == 0; }

int grow_scratch(zipnn_ctx ctx, size_t need)
{
    if (need <= ctx->scratch_cap) return ZIPNN_OK;
    if (ctx->d_scratch) (void)hipFree(ctx->d_scratch);
    ctx->d_scratch = nullptr;
    ctx->scratch_cap = 0;
    size_t cap = need + need / 4;
    if (hipMalloc(&ctx->d_scratch, cap) != hipSuccess) {
        ctx->d_scratch = nullptr;
        return ZIPNN_E_NOMEM;
    }
    ctx->scratch_cap = cap;
    return ZIPNN_OK;
}

int grow_pinned(zipnn_ctx ctx, size_t n)
{
    if (n <= ctx->h_total_cap) return ZIPNN_OK;
    if (ctx->h_total) (void)hipHostFree(ctx->h_total);
    ctx->h_total = nullptr;
    ctx->h_total_cap = 0;
    if (hipHostMalloc((void**)&ctx->h_total, n * sizeof(uint64_t), hipHostMallocDefault) != hipSuccess) return ZIPNN_E_NOMEM;
    ctx->h_total_cap = n;
    return ZIPNN_OK;
}

EncParams make_params(int dtype, const zipnn_params& p)
{
    EncParams e;
    e.dtype = uint32_t(dtype);
    e.B = uint32_t(dtype_bytes(dtype));
    e.chunk = p.chunk_bytes;
    e.S = p.substream_syms;
    e.g = p.group;
    e.L = p.max_code_len;
    e.flags = 0;
    for (int k = 0; k < 4; k++) e.policy[k] = uint32_t(k) < e.B ? p.policy[k] : 0;
    return e;
}

size_t align256(size_t v) { return (v + 255) & ~size_t(255); }

}  // namespace

extern "C" {

const char* zipnn_strerror(int code)
{
    switch (code) {
    case ZIPNN_OK: return "ok";
    case ZIPNN_E_INVAL: return "invalid argument";
    case ZIPNN_E_FORMAT: return "not a valid container header";
    case ZIPNN_E_CORRUPT: return "corrupt container";
    case ZIPNN_E_NOSPACE: return "output buffer too small";
    case ZIPNN_E_NOMEM: return "out of memory";
    case ZIPNN_E_HIP: return "HIP runtime error";
    case ZIPNN_E_BUSY: return "not ready";
    default: return "unknown status";
    }
}

int zipnn_ctx_create(int hip_device, zipnn_ctx* out)
{
    if (!out) return ZIPNN_E_INVAL;
    *out = nullptr;
    int n = 0;
    if (hipGetDeviceCount(&n) != hipSuccess || hip_device < 0 || hip_device >= n) return ZIPNN_E_INVAL;
    zipnn_ctx ctx = new (std::nothrow) zipnn_ctx_s;
    if (!ctx) return ZIPNN_E_NOMEM;
    ctx->device = hip_device;
    DeviceGuard g(hip_device);
    if (hipMalloc((void**)&ctx->d_status, sizeof(int)) != hipSuccess ||
        hipHostMalloc((void**)&ctx->h_status, sizeof(int), hipHostMallocDefault) != hipSuccess ||
        grow_pinned(ctx, 64) != ZIPNN_OK) {
        zipnn_ctx_destroy(ctx);
        return ZIPNN_E_NOMEM;
    }
    if (hipMemset(ctx->d_status, 0, sizeof(int)) != hipSuccess || hipDeviceSynchronize() != hipSuccess) {
        zipnn_ctx_destroy(ctx);
        return ZIPNN_E_HIP;
    }
    ctx->dec_grid = decode_grid_size(hip_device);
    *out = ctx;
    return ZIPNN_OK;
}

void zipnn_ctx_destroy(zipnn_ctx ctx)
{
    if (!ctx) return;
    {
        DeviceGuard g(ctx->device);
        (void)hipDeviceSynchronize();
        if (ctx->d_status) (void)hipFree(ctx->d_status);
        if (ctx->h_status) (void)hipHostFree(ctx->h_status);
        if (ctx->h_total) (void)hipHostFree(ctx->h_total);
        if (ctx->d_scratch) (void)hipFree(ctx->d_scratch);
    }
    delete ctx;
}

int zipnn_ctx_status(zipnn_ctx ctx, void* stream, int clear)
{
    if (!ctx) return ZIPNN_E_INVAL;
    DeviceGuard g(ctx->device);
    hipStream_t s = (hipStream_t)stream;
    if (hipMemcpyAsync(ctx->h_status, ctx->d_status, sizeof(int), hipMemcpyDeviceToHost, s) != hipSuccess)
        return ZIPNN_E_HIP;
    if (clear && launch_clear_status(ctx->d_status, s) != hipSuccess) return ZIPNN_E_HIP;
    if (hipStreamSynchronize(s) != hipSuccess) return ZIPNN_E_HIP;
    return *ctx->h_status;
}

void zipnn_default_params(int dtype, zipnn_params* out)
{
    if (!out) return;
    memset(out, 0, sizeof(*out));
    out->chunk_bytes = 256u << 10;
    // S chosen so that a full 256 KiB chunk has 256 sub-streams per stream:
    // one per thread of a decode workgroup
    const int B = dtype_bytes(dtype) ? dtype_bytes(dtype) : 1;
    out->substream_syms = uint16_t((256u << 10) / uint32_t(B) / 256u);
    out->group = 4;
    out->max_code_len = 11;
    for (int k = 0; k < 4; k++) out->policy[k] = ZIPNN_AUTO;
}

int zipnn_check_params(int dtype, const zipnn_params* p)
{
    const int B = dtype_bytes(dtype);
    if (!B || !p) return ZIPNN_E_INVAL;
    if (check_params(B, p->chunk_bytes, p->substream_syms, p->group, p->max_code_len) != ZIPNN_OK)
        return ZIPNN_E_INVAL;
    for (int k = 0; k < B; k++)
        if (p->policy[k] > ZIPNN_RAW) return ZIPNN_E_INVAL;
    return ZIPNN_OK;
}

uint64_t zipnn_compress_bound(int dtype, uint64_t n, const zipnn_params* p)
{
    if (zipnn_check_params(dtype, p) != ZIPNN_OK) return 0;
    const uint64_t B = uint64_t(dtype_bytes(dtype));
    const uint64_t E = p->chunk_bytes / B;
    const uint64_t nc = (n + E - 1) / E;
    const uint64_t W = (E + p->substream_syms - 1) / p->substream_syms;
    // AUTO never exceeds raw; HUF-forced may reach head + L bits per symbol
    // plus two words of padding per sub-stream
    const uint64_t per_stream = huf_head(uint32_t(W)) + (E * p->max_code_len + 7) / 8 + 8 * W + 16;
    return 64 + 16 * nc * B + nc * B * (per_stream > E + 16 ? per_stream : E + 16);
}

int zipnn_compress(zipnn_ctx ctx, const void* src, int dtype, uint64_t n, const void* base, const zipnn_params* p,
                   void* dst, uint64_t dst_cap, uint64_t* dst_len, void* stream)
{
    if (!ctx || !dst || !dst_len || (!src && n)) return ZIPNN_E_INVAL;
    if (zipnn_check_params(dtype, p) != ZIPNN_OK) return ZIPNN_E_INVAL;
    if (!aligned16(src) || !aligned16(dst) || !aligned16(base)) return ZIPNN_E_INVAL;
    const uint32_t B = uint32_t(dtype_bytes(dtype));
    const uint64_t E = p->chunk_bytes / B;
    const uint64_t nc = (n + E - 1) / E;
    if (nc > 0xFFFFFFFFull) return ZIPNN_E_INVAL;
    if (64 + 16 * nc * B > dst_cap) return ZIPNN_E_NOSPACE;
    std::lock_guard<std::mutex> lk(ctx->mu);
    DeviceGuard g(ctx->device);
    hipStream_t s = (hipStream_t)stream;
    const size_t ne = size_t(nc) * B;
    const size_t off_entries = 0;
    const size_t off_codes = align256(off_entries + ne * sizeof(EncEntry));
    const size_t off_offsets = align256(off_codes + ne * 256 * sizeof(CodeWord));
    const size_t off_nwords = align256(off_offsets + ne * sizeof(uint64_t));
    const size_t off_totals = align256(off_nwords + ne * 64 * sizeof(uint32_t));
    const size_t need = off_totals + 256;
    int rc = grow_scratch(ctx, need);
    if (rc) return rc;
    uint8_t* sc = (uint8_t*)ctx->d_scratch;
    EncEntry* entries = (EncEntry*)(sc + off_entries);
    CodeWord* codes = (CodeWord*)(sc + off_codes);
    uint64_t* offsets = (uint64_t*)(sc + off_offsets);
    uint32_t* nwords = (uint32_t*)(sc + off_nwords);
    uint64_t* totals = (uint64_t*)(sc + off_totals);
    EncParams ep = make_params(dtype, *p);
    ep.flags = base ? kFlagDelta : 0;
    EncDesc one;
    one.src = (const uint8_t*)src;
    one.base = (const uint8_t*)base;
    one.dst = (uint8_t*)dst;
    one.dst_cap = dst_cap;
    one.n = n;
    one.chunk0 = 0;
    one.n_chunks = uint32_t(nc);
    if (launch_analyze(one, nullptr, 1, nullptr, uint32_t(nc), ep, entries, codes, nwords, s) != hipSuccess ||
        launch_place(one, nullptr, 1, ep, entries, offsets, totals, s) != hipSuccess ||
        launch_pack(one, nullptr, 1, nullptr, uint32_t(nc), ep, entries, codes, offsets, totals, nwords, s) !=
            hipSuccess ||
        hipMemcpyAsync(ctx->h_total, totals, sizeof(uint64_t), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
        return ZIPNN_E_HIP;
    const uint64_t total = ctx->h_total[0];
    if (total > dst_cap) return ZIPNN_E_NOSPACE;
    *dst_len = total;
    return ZIPNN_OK;
}

static int decompress_common(zipnn_ctx ctx, const uint32_t* hdr_words, const void* src, uint64_t src_len,
                             const void* base, void* dst, uint64_t dst_cap, hipStream_t s)
{
    Header h;
    int rc = parse_header(hdr_words, src_len, h);
    if (rc) return rc;
    const bool delta = (h.flags & kFlagDelta) != 0;
    if (delta != (base != nullptr)) return ZIPNN_E_INVAL;
    if (h.n * h.B > dst_cap) return ZIPNN_E_NOSPACE;
    if (h.n_chunks == 0) return ZIPNN_OK;
    if (!dst) return ZIPNN_E_INVAL;
    DecDesc one;
    one.src = (const uint8_t*)src;
    one.src_len = src_len;
    one.base = (const uint8_t*)base;
    one.dst = (uint8_t*)dst;
    one.dst_cap = dst_cap;
    if (launch_decode_one(h, one, ctx->d_status, ctx->dec_grid, s) != hipSuccess) return ZIPNN_E_HIP;
    return ZIPNN_OK;
}

int zipnn_decompress(zipnn_ctx ctx, const void* src, uint64_t src_len, const void* base, void* dst, uint64_t dst_cap,
                     void* stream)
{
    if (!ctx || !src) return ZIPNN_E_INVAL;
    if (src_len < 64) return ZIPNN_E_FORMAT;
    if (!aligned16(src) || !aligned16(dst) || !aligned16(base)) return ZIPNN_E_INVAL;
    std::lock_guard<std::mutex> lk(ctx->mu);
    DeviceGuard g(ctx->device);
    hipStream_t s = (hipStream_t)stream;
    // the kernel is chosen from the header: read its 64 bytes (stream-ordered)
    if (hipMemcpyAsync(ctx->h_total, src, 64, hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
        return ZIPNN_E_HIP;
    uint32_t w[16];
    memcpy(w, ctx->h_total, 64);
    return decompress_common(ctx, w, src, src_len, base, dst, dst_cap, s);
}

int zipnn_decompress_async(zipnn_ctx ctx, const void* header_host, const void* src, uint64_t src_len,
                           const void* base, void* dst, uint64_t dst_cap, void* stream)
{
    if (!ctx || !src || !header_host) return ZIPNN_E_INVAL;
    if (src_len < 64) return ZIPNN_E_FORMAT;
    if (!aligned16(src) || !aligned16(dst) || !aligned16(base)) return ZIPNN_E_INVAL;
    DeviceGuard g(ctx->device);
    uint32_t w[16];
    memcpy(w, header_host, 64);
    return decompress_common(ctx, w, src, src_len, base, dst, dst_cap, (hipStream_t)stream);
}

int zipnn_inspect(const void* host_buf, uint64_t len, zipnn_info* out)
{
    if (!host_buf || !out) return ZIPNN_E_INVAL;
    memset(out, 0, sizeof(*out));
    if (len < 64) return ZIPNN_E_FORMAT;
    uint32_t w[16];
    memcpy(w, host_buf, 64);
    Header h;
    // the total is checked against the container's own size field here: the
    // caller may pass only the header and the map
    int rc = parse_header(w, ~0ull, h);
    if (rc) return rc;
    const uint64_t map_end = h.payload_base;
    if (len < map_end) return ZIPNN_E_FORMAT;
    const uint8_t* b = (const uint8_t*)host_buf;
    uint64_t cur = 0;
    for (uint64_t c = 0; c < h.n_chunks; c++) {
        const uint64_t m = h.n - c * h.E < h.E ? h.n - c * h.E : h.E;
        const uint32_t W = uint32_t((m + h.S - 1) / h.S);
        for (uint32_t k = 0; k < h.B; k++) {
            const uint8_t* e = b + 64 + 16 * (c * h.B + k);
            uint64_t off;
            uint32_t bytes;
            memcpy(&off, e, 8);
            memcpy(&bytes, e + 8, 4);
            const uint32_t mode = e[12], rle = e[13];
            if (e[14] || e[15] || mode > 2 || off != cur) return ZIPNN_E_CORRUPT;
            if (mode == kModeRaw && (bytes != m || rle)) return ZIPNN_E_CORRUPT;
            if (mode == kModeRle && bytes) return ZIPNN_E_CORRUPT;
            if (mode == kModeHuf && (bytes < huf_head(W) + (m + 7) / 8 || rle)) return ZIPNN_E_CORRUPT;
            cur += align16(bytes);
            out->bytes_by_mode[mode] += bytes;
            out->entries_by_mode[mode] += 1;
        }
    }
    if (h.payload_base + cur != h.total) return ZIPNN_E_CORRUPT;
    out->dtype = int(h.dtype);
    out->B = int(h.B);
    out->n_elems = h.n;
    out->total_bytes = h.total;
    out->n_chunks = h.n_chunks;
    out->chunk_bytes = h.chunk;
    out->S = h.S;
    out->g = h.g;
    out->L = h.L;
    out->is_delta = (h.flags & kFlagDelta) ? 1 : 0;
    return ZIPNN_OK;
}

}  // extern "C"
