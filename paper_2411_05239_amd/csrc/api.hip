// Host runtime behind include/zipnn.h: contexts, argument checks, scratch
// management, kernel launches and host-side container inspection.
#include <algorithm>
#include <map>
#include <mutex>
#include <new>
#include <string.h>
#include <tuple>
#include <vector>

#include "zipnn_internal.h"

using namespace zipnn;

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
    size_t cap = need + std::min(need / 4, size_t(256) << 20);   // room to grow, at most 256 MiB
    if (dev_malloc((void**)&ctx->d_scratch, cap) != hipSuccess) {
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
    if (host_malloc((void**)&ctx->h_total, n * sizeof(uint64_t)) != hipSuccess) return ZIPNN_E_NOMEM;
    ctx->h_total_cap = n;
    return ZIPNN_OK;
}

// delta: some tensor of the launch has an XOR base (the analysis then runs
// its instance tuned for deltas; headers take the delta flag per tensor)
EncParams make_params(int dtype, const zipnn_params& p, bool delta)
{
    EncParams e;
    e.dtype = uint32_t(dtype);
    e.B = uint32_t(dtype_bytes(dtype));
    e.chunk = p.chunk_bytes;
    e.S = p.substream_syms;
    e.g = p.group;
    e.L = p.max_code_len;
    e.flags = (p.exponent ? kFlagExp : 0u) | (delta ? kFlagDelta : 0u);
    e.skip = p.probe_skip;
    for (int k = 0; k < 4; k++) e.policy[k] = uint32_t(k) < e.B ? p.policy[k] : 0;
    e.stage = nullptr;
    e.stage_chunk = e.stage_lg = e.stage_bm = 0;
    return e;
}

// Staged packing (the analysis skips its second pass over the data; the
// packer writes into staging slots and a compaction places the payloads) for
// launches with an XOR base, whose containers are small next to the bytes
// each pass reads; its slots take about L/8 of the input.  Up to this many
// bytes; beyond, or when the slots cannot be allocated, the exact path.
constexpr size_t kStageMax = size_t(64) << 30;

static size_t stage_bytes_of(bool any_base, uint64_t total_chunks, int dtype, const zipnn_params& p)
{
    if (!any_base) return 0;
    const uint32_t B = uint32_t(dtype_bytes(dtype));
    const StageLayout sl = stage_layout(p.chunk_bytes, B, p.substream_syms, p.group, p.max_code_len);
    const size_t bytes = size_t(total_chunks) * B * sl.chunk;
    return bytes <= kStageMax ? bytes : 0;
}

static void set_stage(EncParams& ep, uint8_t* stage, int dtype, const zipnn_params& p)
{
    const StageLayout sl = stage_layout(p.chunk_bytes, uint32_t(dtype_bytes(dtype)), p.substream_syms, p.group,
                                        p.max_code_len);
    ep.stage = stage;
    ep.stage_chunk = sl.chunk;
    ep.stage_lg = sl.lg;
    ep.stage_bm = sl.bm;
}

size_t align256(size_t v) { return (v + 255) & ~size_t(255); }

// The fixed scratch of zipnn_compress_noalloc: one array in every device's
// memory, held until the process ends.  Its name is a host-side stand-in:
// host code uses only the device address that hipGetSymbolAddress returns
// for the current device, kept per device below.
constexpr size_t kFixedScratch = ZIPNN_NOALLOC_SCRATCH_BYTES;
static __device__ __align__(256) uint8_t scratch[kFixedScratch];
constexpr int kMaxDevices = 64;
std::mutex g_fixed_mu;                     // guards g_fixed_ptr; serialises zipnn_compress_noalloc
void* g_fixed_ptr[kMaxDevices] = {};       // device address of `scratch` on each device

// Once per device, with that device current: look up the array's address.
int fixed_scratch_for(int dev, void** out)
{
    if (dev < 0 || dev >= kMaxDevices) return ZIPNN_E_INVAL;
    std::lock_guard<std::mutex> lk(g_fixed_mu);
    if (!g_fixed_ptr[dev]) {
        void* ptr = nullptr;
        if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return ZIPNN_E_HIP;
        g_fixed_ptr[dev] = ptr;
    }
    *out = g_fixed_ptr[dev];
    return ZIPNN_OK;
}

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
    case ZIPNN_E_TOOBIG: return "input needs more than the fixed scratch of the allocation-free entry point";
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
    if (dev_malloc((void**)&ctx->d_status, sizeof(int)) != hipSuccess ||
        host_malloc((void**)&ctx->h_status, sizeof(int)) != hipSuccess ||
        grow_pinned(ctx, 64) != ZIPNN_OK) {
        zipnn_ctx_destroy(ctx);
        return ZIPNN_E_NOMEM;
    }
    if (hipMemset(ctx->d_status, 0, sizeof(int)) != hipSuccess || hipDeviceSynchronize() != hipSuccess) {
        zipnn_ctx_destroy(ctx);
        return ZIPNN_E_HIP;
    }
    // the fixed scratch's address on this device (checked; without it only
    // zipnn_compress_noalloc is unavailable, and it says so)
    if (fixed_scratch_for(hip_device, &ctx->fixed_scratch) != ZIPNN_OK) ctx->fixed_scratch = nullptr;
    for (uint32_t B : {1u, 2u, 4u})
        for (uint32_t G : {2u, 4u, 8u})
            for (int d = 0; d < 2; d++)
                for (int z = 0; z < 2; z++) {
                    const DecClass k{B, G, d != 0, z != 0};
                    ctx->dec_grid[dec_class_index(k)] = decode_grid_size(hip_device, k);
                }
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
        if (p->policy[k] > ZIPNN_ZG) return ZIPNN_E_INVAL;
    if (p->reserved[0] || p->reserved[1]) return ZIPNN_E_INVAL;
    if (p->exponent > 1 || (p->exponent && dtype != ZIPNN_BF16 && dtype != ZIPNN_FP32)) return ZIPNN_E_INVAL;
    return ZIPNN_OK;
}

uint64_t zipnn_compress_bound(int dtype, uint64_t n, const zipnn_params* p)
{
    if (zipnn_check_params(dtype, p) != ZIPNN_OK) return 0;
    const uint64_t B = uint64_t(dtype_bytes(dtype));
    const uint64_t E = p->chunk_bytes / B;
    const uint64_t nc = (n + E - 1) / E;
    const uint64_t W = (E + p->substream_syms - 1) / p->substream_syms;
    // AUTO never exceeds raw; HUF- or ZG-forced may reach head + a bitmap of
    // one bit per two symbols + L bits per symbol plus two words of padding
    // per sub-stream
    const uint64_t per_stream =
        huf_head(uint32_t(W)) + (E / 16 + 16) + (E * p->max_code_len + 7) / 8 + 8 * W;
    return 64 + kPayAlign + 16 * nc * B + nc * B * ((per_stream > E ? per_stream : E) + kPayAlign);
}

// Encode tensors[0..n) (all of one dtype) into `arena`; offsets_host gets the
// n+1 arena offsets.  Blocking.
static int encode_tensors(zipnn_ctx ctx, int dtype, const zipnn_tensor_in* t, int n, const zipnn_params* p,
                          void* arena, uint64_t cap, uint64_t* offsets_host, hipStream_t s)
{
    if (zipnn_check_params(dtype, p) != ZIPNN_OK || n < 1 || !arena || !offsets_host) return ZIPNN_E_INVAL;
    if (!aligned16(arena)) return ZIPNN_E_INVAL;
    const uint32_t B = uint32_t(dtype_bytes(dtype));
    const uint64_t E = p->chunk_bytes / B;
    uint64_t total_chunks = 0, map_bytes = 0;
    for (int i = 0; i < n; i++) {
        if ((!t[i].src && t[i].n_elems) || !aligned16(t[i].src) || !aligned16(t[i].base)) return ZIPNN_E_INVAL;
        const uint64_t nc = (t[i].n_elems + E - 1) / E;
        total_chunks += nc;
        map_bytes += payload_base_of(nc, B);
    }
    if (total_chunks > 0xFFFFFFFFull) return ZIPNN_E_INVAL;
    if (map_bytes > cap) return ZIPNN_E_NOSPACE;
    std::lock_guard<std::mutex> lk(ctx->mu);
    DeviceGuard g(ctx->device);
    bool any_base = false;
    for (int i = 0; i < n; i++) any_base |= t[i].base != nullptr;
    size_t stage = stage_bytes_of(any_base, total_chunks, dtype, *p);
    EncScratch lay = enc_scratch_layout(size_t(total_chunks) * B, size_t(n), stage);
    int rc = grow_scratch(ctx, lay.need);
    if (rc && stage) {   // no room for the staging slots: the exact path
        stage = 0;
        lay = enc_scratch_layout(size_t(total_chunks) * B, size_t(n));
        rc = grow_scratch(ctx, lay.need);
    }
    if (rc) return rc;
    // host staging (pinned): descriptors, chunk prefix, then the arena offsets
    const size_t stage_bytes = size_t(n) * sizeof(EncDesc) + size_t(n + 1) * sizeof(uint32_t) +
                               size_t(n + 1) * sizeof(uint64_t) + 64;
    rc = grow_pinned(ctx, stage_bytes / sizeof(uint64_t) + 1);
    if (rc) return rc;
    EncDesc* hd = (EncDesc*)ctx->h_total;
    uint32_t* hp = (uint32_t*)(hd + n);
    uint64_t* ho = (uint64_t*)align16(uint64_t(hp + n + 1));
    uint32_t run = 0;
    for (int i = 0; i < n; i++) {
        const uint64_t nc = (t[i].n_elems + E - 1) / E;
        hd[i].src = (const uint8_t*)t[i].src;
        hd[i].base = (const uint8_t*)t[i].base;
        hd[i].dst = nullptr;
        hd[i].dst_cap = 0;
        hd[i].n = t[i].n_elems;
        hd[i].chunk0 = run;
        hd[i].n_chunks = uint32_t(nc);
        hd[i].has_zg = 0;
        hd[i].pad = 0;
        hp[i] = run;
        run += uint32_t(nc);
    }
    hp[n] = run;
    uint8_t* sc = (uint8_t*)ctx->d_scratch;
    EncDesc* d_descs = (EncDesc*)(sc + lay.descs);
    uint32_t* d_prefix = (uint32_t*)(sc + lay.prefix);
    uint64_t* d_aoff = (uint64_t*)(sc + lay.aoff);
    EncParams ep = make_params(dtype, *p, any_base);
    if (stage) set_stage(ep, sc + lay.stage, dtype, *p);
    if (hipMemcpyAsync(d_descs, hd, size_t(n) * sizeof(EncDesc), hipMemcpyHostToDevice, s) != hipSuccess ||
        hipMemcpyAsync(d_prefix, hp, size_t(n + 1) * sizeof(uint32_t), hipMemcpyHostToDevice, s) != hipSuccess ||
        launch_encode(d_descs, n, d_prefix, uint32_t(total_chunks), ep, (uint8_t*)arena, cap,
                      (EncEntry*)(sc + lay.entries), (CodeWord*)(sc + lay.codes), (uint32_t*)(sc + lay.nwords),
                      (uint64_t*)(sc + lay.offsets), (uint64_t*)(sc + lay.totals), d_aoff, s) != hipSuccess ||
        hipMemcpyAsync(ho, d_aoff, size_t(n + 1) * sizeof(uint64_t), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
        return ZIPNN_E_HIP;
    if (ho[n] > cap) return ZIPNN_E_NOSPACE;
    memcpy(offsets_host, ho, size_t(n + 1) * sizeof(uint64_t));
    return ZIPNN_OK;
}

int zipnn_compress(zipnn_ctx ctx, const void* src, int dtype, uint64_t n, const void* base, const zipnn_params* p,
                   void* dst, uint64_t dst_cap, uint64_t* dst_len, void* stream)
{
    if (!ctx || !dst || !dst_len || (!src && n)) return ZIPNN_E_INVAL;
    zipnn_tensor_in t;
    t.src = src;
    t.n_elems = n;
    t.base = base;
    uint64_t off[2];
    const int rc = encode_tensors(ctx, dtype, &t, 1, p, dst, dst_cap, off, (hipStream_t)stream);
    if (rc == ZIPNN_OK) *dst_len = off[1];
    return rc;
}

int zipnn_compress_noalloc(zipnn_ctx ctx, const void* src, int dtype, uint64_t n, const void* base,
                           const zipnn_params* p, void* dst, uint64_t dst_cap, uint64_t* dst_len, void* stream)
{
    if (!ctx || !dst || !dst_len || (!src && n)) return ZIPNN_E_INVAL;
    if (zipnn_check_params(dtype, p) != ZIPNN_OK) return ZIPNN_E_INVAL;
    if (!aligned16(dst) || !aligned16(src) || !aligned16(base)) return ZIPNN_E_INVAL;
    const uint32_t B = uint32_t(dtype_bytes(dtype));
    const uint64_t E = p->chunk_bytes / B;
    const uint64_t nc = (n + E - 1) / E;
    if (payload_base_of(nc, B) > dst_cap) return ZIPNN_E_NOSPACE;
    const EncScratch lay = enc_scratch_layout(size_t(nc) * B, 1);
    if (lay.need > kFixedScratch) return ZIPNN_E_TOOBIG;
    if (!ctx->fixed_scratch) return ZIPNN_E_HIP;
    std::lock_guard<std::mutex> lk(g_fixed_mu);
    DeviceGuard g(ctx->device);
    hipStream_t s = (hipStream_t)stream;
    uint8_t* sc = (uint8_t*)ctx->fixed_scratch;
    EncDesc one;
    one.src = (const uint8_t*)src;
    one.base = (const uint8_t*)base;
    one.dst = nullptr;
    one.dst_cap = 0;
    one.n = n;
    one.chunk0 = 0;
    one.n_chunks = uint32_t(nc);
    one.has_zg = 0;
    one.pad = 0;
    EncDesc* d_descs = (EncDesc*)(sc + lay.descs);
    uint32_t* d_prefix = (uint32_t*)(sc + lay.prefix);
    uint64_t* d_aoff = (uint64_t*)(sc + lay.aoff);
    uint64_t ho[2] = {0, 0};   // the arena offsets come back to the stack
    const EncParams ep = make_params(dtype, *p, one.base != nullptr);
    if (launch_fill_desc(one, uint32_t(nc), d_descs, d_prefix, s) != hipSuccess ||
        launch_encode(d_descs, 1, d_prefix, uint32_t(nc), ep, (uint8_t*)dst, dst_cap, (EncEntry*)(sc + lay.entries),
                      (CodeWord*)(sc + lay.codes), (uint32_t*)(sc + lay.nwords), (uint64_t*)(sc + lay.offsets),
                      (uint64_t*)(sc + lay.totals), d_aoff, s) != hipSuccess ||
        hipMemcpyAsync(ho, d_aoff, sizeof(ho), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
        return ZIPNN_E_HIP;
    if (ho[1] > dst_cap) return ZIPNN_E_NOSPACE;
    *dst_len = ho[1];
    return ZIPNN_OK;
}

int zipnn_compress_batch(zipnn_ctx ctx, int dtype, const zipnn_tensor_in* tensors, int n, const zipnn_params* p,
                         void* arena, uint64_t arena_cap, uint64_t* offsets, void* stream)
{
    if (!ctx || !tensors) return ZIPNN_E_INVAL;
    return encode_tensors(ctx, dtype, tensors, n, p, arena, arena_cap, offsets, (hipStream_t)stream);
}

// ------------------------------------------------------------ prepared encodes

struct zipnn_encoder_s {
    zipnn_ctx ctx = nullptr;
    int n = 0;
    uint64_t cap = 0;
    void* d_mem = nullptr;        // scratch, descriptors and chunk prefix of this batch
    uint64_t* h_offs = nullptr;   // pinned: the n+1 arena offsets of the last run
    hipStream_t capst = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

int zipnn_encoder_create(zipnn_ctx ctx, int dtype, const zipnn_tensor_in* t, int n, const zipnn_params* p,
                         void* arena, uint64_t cap, zipnn_encoder* out)
{
    if (!ctx || !t || !out) return ZIPNN_E_INVAL;
    *out = nullptr;
    if (zipnn_check_params(dtype, p) != ZIPNN_OK || n < 1 || !arena || !aligned16(arena)) return ZIPNN_E_INVAL;
    const uint32_t B = uint32_t(dtype_bytes(dtype));
    const uint64_t E = p->chunk_bytes / B;
    uint64_t total_chunks = 0, map_bytes = 0;
    for (int i = 0; i < n; i++) {
        if ((!t[i].src && t[i].n_elems) || !aligned16(t[i].src) || !aligned16(t[i].base)) return ZIPNN_E_INVAL;
        const uint64_t nc = (t[i].n_elems + E - 1) / E;
        total_chunks += nc;
        map_bytes += payload_base_of(nc, B);
    }
    if (total_chunks > 0xFFFFFFFFull) return ZIPNN_E_INVAL;
    if (map_bytes > cap) return ZIPNN_E_NOSPACE;
    DeviceGuard g(ctx->device);
    zipnn_encoder e = new (std::nothrow) zipnn_encoder_s;
    if (!e) return ZIPNN_E_NOMEM;
    e->ctx = ctx;
    e->n = n;
    e->cap = cap;
    bool any_base = false;
    for (int i = 0; i < n; i++) any_base |= t[i].base != nullptr;
    size_t stage = stage_bytes_of(any_base, total_chunks, dtype, *p);
    EncScratch lay = enc_scratch_layout(size_t(total_chunks) * B, size_t(n), stage);
    std::vector<EncDesc> hd(static_cast<size_t>(n));
    std::vector<uint32_t> hp(static_cast<size_t>(n) + 1);
    uint32_t run = 0;
    for (int i = 0; i < n; i++) {
        const uint64_t nc = (t[i].n_elems + E - 1) / E;
        hd[size_t(i)] = EncDesc{(const uint8_t*)t[i].src, (const uint8_t*)t[i].base, nullptr, 0, t[i].n_elems, run,
                                uint32_t(nc), 0, 0};
        hp[size_t(i)] = run;
        run += uint32_t(nc);
    }
    hp[size_t(n)] = run;
    if (dev_malloc((void**)&e->d_mem, lay.need) != hipSuccess && stage) {   // no room for the staging slots
        e->d_mem = nullptr;
        stage = 0;
        lay = enc_scratch_layout(size_t(total_chunks) * B, size_t(n));
        if (dev_malloc((void**)&e->d_mem, lay.need) != hipSuccess) e->d_mem = nullptr;
    }
    if (!e->d_mem ||
        host_malloc((void**)&e->h_offs, size_t(n + 1) * sizeof(uint64_t)) != hipSuccess) {
        zipnn_encoder_destroy(e);
        return ZIPNN_E_NOMEM;
    }
    uint8_t* sc = (uint8_t*)e->d_mem;
    EncDesc* d_descs = (EncDesc*)(sc + lay.descs);
    uint32_t* d_prefix = (uint32_t*)(sc + lay.prefix);
    uint64_t* d_aoff = (uint64_t*)(sc + lay.aoff);
    if (hipMemcpy(d_descs, hd.data(), hd.size() * sizeof(EncDesc), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(d_prefix, hp.data(), hp.size() * sizeof(uint32_t), hipMemcpyHostToDevice) != hipSuccess) {
        zipnn_encoder_destroy(e);
        return ZIPNN_E_HIP;
    }
    // capture the launches and the copy of the offsets once; every run replays them
    EncParams ep = make_params(dtype, *p, any_base);
    if (stage) set_stage(ep, sc + lay.stage, dtype, *p);
    if (hipStreamCreateWithFlags(&e->capst, hipStreamNonBlocking) != hipSuccess ||
        hipStreamBeginCapture(e->capst, hipStreamCaptureModeThreadLocal) != hipSuccess) {
        zipnn_encoder_destroy(e);
        return ZIPNN_E_HIP;
    }
    hipError_t le = launch_encode(d_descs, n, d_prefix, uint32_t(total_chunks), ep, (uint8_t*)arena, cap,
                                  (EncEntry*)(sc + lay.entries), (CodeWord*)(sc + lay.codes),
                                  (uint32_t*)(sc + lay.nwords), (uint64_t*)(sc + lay.offsets),
                                  (uint64_t*)(sc + lay.totals), d_aoff, e->capst);
    if (le == hipSuccess)
        le = hipMemcpyAsync(e->h_offs, d_aoff, size_t(n + 1) * sizeof(uint64_t), hipMemcpyDeviceToHost, e->capst);
    const hipError_t ce = hipStreamEndCapture(e->capst, &e->graph);
    if (le != hipSuccess || ce != hipSuccess || hipGraphInstantiate(&e->exec, e->graph, nullptr, nullptr, 0) != hipSuccess) {
        zipnn_encoder_destroy(e);
        return ZIPNN_E_HIP;
    }
    *out = e;
    return ZIPNN_OK;
}

int zipnn_encoder_run(zipnn_encoder e, void* stream, uint64_t* offsets)
{
    if (!e || !offsets) return ZIPNN_E_INVAL;
    DeviceGuard g(e->ctx->device);
    hipStream_t s = (hipStream_t)stream;
    if (hipGraphLaunch(e->exec, s) != hipSuccess || hipStreamSynchronize(s) != hipSuccess) return ZIPNN_E_HIP;
    if (e->h_offs[e->n] > e->cap) return ZIPNN_E_NOSPACE;
    memcpy(offsets, e->h_offs, size_t(e->n + 1) * sizeof(uint64_t));
    return ZIPNN_OK;
}

void zipnn_encoder_destroy(zipnn_encoder e)
{
    if (!e) return;
    DeviceGuard g(e->ctx->device);
    (void)hipDeviceSynchronize();
    if (e->exec) (void)hipGraphExecDestroy(e->exec);
    if (e->graph) (void)hipGraphDestroy(e->graph);
    if (e->capst) (void)hipStreamDestroy(e->capst);
    if (e->d_mem) (void)hipFree(e->d_mem);
    if (e->h_offs) (void)hipHostFree(e->h_offs);
    delete e;
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
    one.c_begin = 0;
    one.c_end = kAllChunks;
    one.status = nullptr;
    // no more workgroups than items: a small tensor does not dispatch the
    // whole persistent grid
    const uint64_t items = plan_items(h, 0, kAllChunks).items;
    const int grid = int(std::min<uint64_t>(uint64_t(ctx->dec_grid[dec_class_index(dec_class(h))]),
                                            std::max<uint64_t>(items, 1)));
    if (launch_decode_one(h, one, ctx->d_status, grid, s) != hipSuccess) return ZIPNN_E_HIP;
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

// ------------------------------------------------------------ prepared batches

struct zipnn_batch_s {
    struct Class {
        DecClass k;
        int n;
        DecDesc* d_descs;
        uint64_t* d_prefix;
    };
    zipnn_ctx ctx = nullptr;
    std::vector<Class> classes;
    void* d_mem = nullptr;
    hipStream_t cap = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

static hipError_t batch_launch(zipnn_batch b, hipStream_t s)
{
    for (auto& c : b->classes) {
        hipError_t e = launch_decode_batch(c.k, c.d_descs, c.n, c.d_prefix, b->ctx->d_status,
                                           b->ctx->dec_grid[dec_class_index(c.k)], s);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

int zipnn_batch_create(zipnn_ctx ctx, const void* arena, const uint64_t* offsets, int n, void* const* dst,
                       const uint64_t* dst_cap, const void* const* base, zipnn_batch* out)
{
    if (!ctx || !arena || !offsets || !dst || !dst_cap || !out || n < 1) return ZIPNN_E_INVAL;
    *out = nullptr;
    if (!aligned16(arena)) return ZIPNN_E_INVAL;
    for (int i = 0; i < n; i++) {
        if ((offsets[i] & 15) || offsets[i + 1] < offsets[i] + 64) return ZIPNN_E_INVAL;
        if (!aligned16(dst[i]) || (base && !aligned16(base[i]))) return ZIPNN_E_INVAL;
    }
    std::lock_guard<std::mutex> lk(ctx->mu);
    DeviceGuard g(ctx->device);
    // headers -> host, in one gather
    int rc = grow_scratch(ctx, size_t(n + 1) * 8 + size_t(n) * 64 + 256);
    if (rc) return rc;
    rc = grow_pinned(ctx, size_t(n) * 8 + 8);
    if (rc) return rc;
    uint64_t* d_offs = (uint64_t*)ctx->d_scratch;
    uint8_t* d_hdr = (uint8_t*)ctx->d_scratch + align256(size_t(n + 1) * 8);
    hipStream_t s0 = nullptr;
    if (hipMemcpyAsync(d_offs, offsets, size_t(n + 1) * 8, hipMemcpyHostToDevice, s0) != hipSuccess ||
        launch_gather_headers((const uint8_t*)arena, d_offs, n, d_hdr, s0) != hipSuccess ||
        hipMemcpyAsync(ctx->h_total, d_hdr, size_t(n) * 64, hipMemcpyDeviceToHost, s0) != hipSuccess ||
        hipStreamSynchronize(s0) != hipSuccess)
        return ZIPNN_E_HIP;
    // group the tensors by kernel class (B, g, delta, zg)
    std::map<std::tuple<uint32_t, uint32_t, bool, bool>, std::vector<DecDesc>> groups;
    for (int i = 0; i < n; i++) {
        Header h;
        rc = parse_header((const uint32_t*)((const uint8_t*)ctx->h_total + 64 * size_t(i)), offsets[i + 1] - offsets[i],
                          h);
        if (rc) return rc;
        const bool delta = (h.flags & kFlagDelta) != 0;
        const void* bi = base ? base[i] : nullptr;
        if (delta != (bi != nullptr)) return ZIPNN_E_INVAL;
        if (h.n * h.B > dst_cap[i]) return ZIPNN_E_NOSPACE;
        if (h.n_chunks == 0) continue;
        DecDesc d;
        d.src = (const uint8_t*)arena + offsets[i];
        d.src_len = offsets[i + 1] - offsets[i];
        d.base = (const uint8_t*)bi;
        d.dst = (uint8_t*)dst[i];
        d.dst_cap = dst_cap[i];
        d.c_begin = 0;
        d.c_end = kAllChunks;
        d.status = nullptr;
        groups[std::make_tuple(h.B, h.g, delta, (h.flags & kFlagZg) != 0)].push_back(d);
    }
    zipnn_batch b = new (std::nothrow) zipnn_batch_s;
    if (!b) return ZIPNN_E_NOMEM;
    b->ctx = ctx;
    size_t bytes = 0;
    for (auto& kv : groups) bytes += align256(kv.second.size() * sizeof(DecDesc)) + align256((kv.second.size() + 2) * 8);
    if (bytes && dev_malloc((void**)&b->d_mem, bytes) != hipSuccess) {
        delete b;
        return ZIPNN_E_NOMEM;
    }
    size_t off = 0;
    for (auto& kv : groups) {
        zipnn_batch_s::Class c;
        c.k = DecClass{std::get<0>(kv.first), std::get<1>(kv.first), std::get<2>(kv.first), std::get<3>(kv.first)};
        c.n = int(kv.second.size());
        c.d_descs = (DecDesc*)((uint8_t*)b->d_mem + off);
        off += align256(kv.second.size() * sizeof(DecDesc));
        c.d_prefix = (uint64_t*)((uint8_t*)b->d_mem + off);
        off += align256((kv.second.size() + 2) * 8);
        if (hipMemcpy(c.d_descs, kv.second.data(), kv.second.size() * sizeof(DecDesc), hipMemcpyHostToDevice) !=
            hipSuccess) {
            zipnn_batch_destroy(b);
            return ZIPNN_E_HIP;
        }
        b->classes.push_back(c);
    }
    // capture the launches once; every decompress replays the graph
    if (hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking) != hipSuccess ||
        hipStreamBeginCapture(b->cap, hipStreamCaptureModeThreadLocal) != hipSuccess) {
        zipnn_batch_destroy(b);
        return ZIPNN_E_HIP;
    }
    const hipError_t le = batch_launch(b, b->cap);
    const hipError_t ce = hipStreamEndCapture(b->cap, &b->graph);
    if (le != hipSuccess || ce != hipSuccess || hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0) != hipSuccess) {
        zipnn_batch_destroy(b);
        return ZIPNN_E_HIP;
    }
    *out = b;
    return ZIPNN_OK;
}

int zipnn_batch_decompress(zipnn_batch b, void* stream)
{
    if (!b) return ZIPNN_E_INVAL;
    DeviceGuard g(b->ctx->device);
    if (b->classes.empty()) return ZIPNN_OK;
    return hipGraphLaunch(b->exec, (hipStream_t)stream) == hipSuccess ? ZIPNN_OK : ZIPNN_E_HIP;
}

void zipnn_batch_destroy(zipnn_batch b)
{
    if (!b) return;
    DeviceGuard g(b->ctx->device);
    (void)hipDeviceSynchronize();
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    if (b->cap) (void)hipStreamDestroy(b->cap);
    if (b->d_mem) (void)hipFree(b->d_mem);
    delete b;
}

int zipnn_decompress_batch(zipnn_ctx ctx, const void* arena, const uint64_t* offsets, int n, void* const* dst,
                           const uint64_t* dst_cap, const void* const* base, void* stream)
{
    zipnn_batch b = nullptr;
    int rc = zipnn_batch_create(ctx, arena, offsets, n, dst, dst_cap, base, &b);
    if (rc) return rc;
    rc = zipnn_batch_decompress(b, stream);
    if (rc == ZIPNN_OK && hipStreamSynchronize((hipStream_t)stream) != hipSuccess) rc = ZIPNN_E_HIP;
    zipnn_batch_destroy(b);
    return rc;
}

// ------------------------------------------------------------ autotuner

int zipnn_autotune(zipnn_ctx ctx, int dtype, const zipnn_tensor_in* tensors, int n, const zipnn_tune_config* cfg,
                   zipnn_params* best, zipnn_tune_entry* entries, int max_entries, int* n_entries)
{
    const int B = dtype_bytes(dtype);
    if (!ctx || !tensors || n < 1 || !best || !B) return ZIPNN_E_INVAL;
    zipnn_tune_config c = {};
    if (cfg) c = *cfg;
    if (c.max_ratio_loss < 0 || c.tie < 0 || c.repeats < 0) return ZIPNN_E_INVAL;
    if (!c.sample_bytes) c.sample_bytes = 1ull << 30;
    if (!c.min_chunk && !c.max_chunk) {
        c.min_chunk = 64u << 10;
        c.max_chunk = 1u << 20;
    }
    if (!pow2(c.min_chunk) || !pow2(c.max_chunk) || c.min_chunk > c.max_chunk || c.min_chunk < kMinChunk ||
        c.max_chunk > kMaxChunk)
        return ZIPNN_E_INVAL;
    if (!c.repeats) c.repeats = 7;
    if (c.tie == 0) c.tie = 0.02;
    // the sample, stratified by size class (tensors of equal length, e.g. the
    // q projections of every layer): each class gets its share of
    // sample_bytes, filled with its tensors in order, whole, the last one cut
    // to the remaining share (at least one largest chunk); every class is in
    // it, and the tensors keep their real lengths, so the chunk and work-item
    // counts per tensor are the checkpoint's own
    uint64_t total = 0;
    for (int i = 0; i < n; i++) total += tensors[i].n_elems * uint64_t(B);
    if (!total) return ZIPNN_E_INVAL;
    std::vector<uint64_t> take(size_t(n), 0);
    if (total <= c.sample_bytes) {
        for (int i = 0; i < n; i++) take[size_t(i)] = tensors[i].n_elems;
    } else {
        std::vector<uint64_t> sizes;   // the classes in order of first appearance
        for (int i = 0; i < n; i++)
            if (tensors[i].n_elems && std::find(sizes.begin(), sizes.end(), tensors[i].n_elems) == sizes.end())
                sizes.push_back(tensors[i].n_elems);
        for (const uint64_t len : sizes) {
            uint64_t cls = 0;
            for (int i = 0; i < n; i++)
                if (tensors[i].n_elems == len) cls += len;
            uint64_t left = uint64_t(((unsigned __int128)cls * c.sample_bytes + total - 1) / total) / uint64_t(B);
            for (int i = 0; i < n && left; i++) {
                if (tensors[i].n_elems != len) continue;
                const uint64_t k = std::min<uint64_t>(len, std::max<uint64_t>(left, c.max_chunk / uint32_t(B)));
                take[size_t(i)] = k;
                left -= std::min(left, k);
            }
        }
    }
    std::vector<zipnn_tensor_in> smp;
    uint64_t sbytes = 0;
    for (int i = 0; i < n; i++) {
        if (!take[size_t(i)]) continue;
        zipnn_tensor_in t = tensors[i];
        t.n_elems = take[size_t(i)];
        smp.push_back(t);
        sbytes += t.n_elems * uint64_t(B);
    }
    // candidate formats: chunk size x sub-stream length, with 256 to 2048
    // sub-streams per chunk (at least a decode workgroup's four lane groups)
    std::vector<zipnn_params> cands;
    for (uint32_t chunk = c.min_chunk; chunk <= c.max_chunk; chunk <<= 1) {
        const uint32_t E = chunk / uint32_t(B);
        for (uint32_t div = 256; div <= 2048; div <<= 1) {
            zipnn_params p;
            zipnn_default_params(dtype, &p);
            p.chunk_bytes = chunk;
            p.substream_syms = uint16_t(std::max<uint32_t>(4, E / div));
            for (int k = 0; k < 4; k++) p.policy[k] = c.policy[k];
            if (zipnn_check_params(dtype, &p) == ZIPNN_OK) cands.push_back(p);
        }
    }
    if (cands.empty()) return ZIPNN_E_INVAL;   // e.g. a policy value out of range
    DeviceGuard g(ctx->device);
    uint64_t cap = 0;
    for (const auto& p : cands) {
        uint64_t cb = 0;
        for (const auto& t : smp) cb += zipnn_compress_bound(dtype, t.n_elems, &p) + kPayAlign;
        cap = std::max(cap, cb);
    }
    void* arena = nullptr;
    void* outs = nullptr;
    if (dev_malloc((void**)&arena, cap) != hipSuccess) return ZIPNN_E_NOMEM;
    if (dev_malloc((void**)&outs, align256(sbytes) + 256 * smp.size()) != hipSuccess) {
        (void)hipFree(arena);
        return ZIPNN_E_NOMEM;
    }
    std::vector<void*> dst(smp.size());
    std::vector<uint64_t> caps(smp.size());
    std::vector<const void*> bases(smp.size());
    bool any_base = false;
    {
        uint64_t o = 0;
        for (size_t i = 0; i < smp.size(); i++) {
            dst[i] = (uint8_t*)outs + o;
            caps[i] = smp[i].n_elems * uint64_t(B);
            bases[i] = smp[i].base;
            any_base |= smp[i].base != nullptr;
            o += align256(caps[i]);
        }
    }
    hipStream_t s = nullptr;
    hipEvent_t e0, e1;
    (void)hipEventCreate(&e0);
    (void)hipEventCreate(&e1);
    std::vector<zipnn_tune_entry> res;
    int rc = ZIPNN_OK;
    std::vector<uint64_t> offs(smp.size() + 1);
    std::vector<float> times(size_t(c.repeats));
    for (const auto& p : cands) {
        (void)hipEventRecord(e0, s);
        rc = zipnn_compress_batch(ctx, dtype, smp.data(), int(smp.size()), &p, arena, cap, offs.data(), s);
        (void)hipEventRecord(e1, s);
        if (rc) break;
        (void)hipEventSynchronize(e1);
        float enc_ms = 0;
        (void)hipEventElapsedTime(&enc_ms, e0, e1);
        zipnn_batch b = nullptr;
        rc = zipnn_batch_create(ctx, arena, offs.data(), int(smp.size()), dst.data(), caps.data(),
                                any_base ? bases.data() : nullptr, &b);
        if (rc) break;
        (void)zipnn_batch_decompress(b, s);   // warm-up
        for (int r = 0; r < c.repeats; r++) {
            (void)hipEventRecord(e0, s);
            (void)zipnn_batch_decompress(b, s);
            (void)hipEventRecord(e1, s);
            (void)hipEventSynchronize(e1);
            (void)hipEventElapsedTime(&times[size_t(r)], e0, e1);
        }
        zipnn_batch_destroy(b);
        std::sort(times.begin(), times.end());
        const float med = times[times.size() / 2];
        zipnn_tune_entry te;
        te.params = p;
        te.ratio = double(offs.back()) / double(sbytes);
        te.decode_gbps = double(sbytes) / (double(med) * 1e6);
        te.encode_gbps = double(sbytes) / (double(enc_ms) * 1e6);
        res.push_back(te);
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    (void)hipFree(arena);
    (void)hipFree(outs);
    if (rc) return rc;
    if (zipnn_ctx_status(ctx, nullptr, 1) != ZIPNN_OK) return ZIPNN_E_CORRUPT;
    // within the ratio loss: the fastest decode sets the bar; every candidate
    // within `tie` of it ties; the smallest chunk wins, then the best ratio
    double best_ratio = 1e30;
    for (const auto& r : res) best_ratio = std::min(best_ratio, r.ratio);
    double fastest = 0;
    for (const auto& r : res)
        if (r.ratio <= best_ratio * (1.0 + c.max_ratio_loss)) fastest = std::max(fastest, r.decode_gbps);
    int pick = -1;
    for (size_t i = 0; i < res.size(); i++) {
        const auto& r = res[i];
        if (r.ratio > best_ratio * (1.0 + c.max_ratio_loss) || r.decode_gbps < fastest * (1.0 - c.tie)) continue;
        if (pick < 0 || r.params.chunk_bytes < res[pick].params.chunk_bytes ||
            (r.params.chunk_bytes == res[pick].params.chunk_bytes && r.ratio < res[pick].ratio))
            pick = int(i);
    }
    *best = res[size_t(pick)].params;
    if (n_entries) *n_entries = int(res.size());
    if (entries)
        for (int i = 0; i < std::min(max_entries, int(res.size())); i++) entries[i] = res[size_t(i)];
    return ZIPNN_OK;
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
    const uint64_t map_end = 64 + 16ull * h.n_chunks * h.B;
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
            if (e[14] || e[15] || mode > 3 || off != cur) return ZIPNN_E_CORRUPT;
            if (mode == kModeRaw && (bytes != m || rle)) return ZIPNN_E_CORRUPT;
            if (mode == kModeRle && bytes) return ZIPNN_E_CORRUPT;
            if (mode == kModeHuf && (bytes < huf_head(W) + (m + 7) / 8 || rle)) return ZIPNN_E_CORRUPT;
            if (mode == kModeZg && bytes < huf_head(W) + zg_bitmap(uint32_t(m), h.g)) return ZIPNN_E_CORRUPT;
            cur += align_pay(bytes);
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
