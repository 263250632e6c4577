// Decompression server behind the zipnn_server_* calls of include/zipnn.h:
// resident containers, an output pool in device memory with first-fit
// allocation, admission in arrival order by free pool bytes, and a scheduler
// thread that packs chunk ranges of the admitted requests into decode
// iterations (continuous batching).  Chunks are independent given the map
// (paper §V-A), so the bytes of a request do not depend on what it was
// batched with; iterations go to one stream, two in flight.
#include <string.h>
#include <time.h>

#include <algorithm>
#include <atomic>
#include <condition_variable>
#include <deque>
#include <map>
#include <mutex>
#include <new>
#include <thread>
#include <tuple>
#include <unordered_map>
#include <vector>

#include "zipnn_internal.h"

using namespace zipnn;

namespace {

constexpr int kIterDepth = 2;            // iterations in flight
constexpr uint64_t kPoolAlign = 256;
constexpr uint32_t kDefaultChunksPerIter = 2048;
// The scheduler polls this long before it sleeps: a sleeping scheduler costs
// each arrival a thread wake-up (tens of microseconds); at 100 requests/s
// only gaps longer than this (e^-5 of them) pay it.
constexpr double kIdleSpinSeconds = 50e-3;
double now_s()
{
    timespec ts;
    clock_gettime(CLOCK_MONOTONIC, &ts);
    return double(ts.tv_sec) + 1e-9 * double(ts.tv_nsec);
}

uint64_t round_up(uint64_t v, uint64_t a) { return (v + a - 1) / a * a; }

struct Entry {
    const uint8_t* src;
    uint64_t len;
    const uint8_t* base;
    Header h;
};

enum { kPending = 0, kActive = 1, kDone = 2 };

struct Req {
    uint32_t handle = 0;
    int state = kPending;
    int status = ZIPNN_OK;
    uint64_t off = 0;        // output offset in the pool
    uint64_t bytes = 0;      // output bytes (n * B)
    uint64_t held = 0;       // pool bytes held
    uint32_t next = 0;       // first chunk not yet launched
    uint32_t n_chunks = 0;
    bool launched = false;
    zipnn_timing t = {};
};

// One decode iteration: descriptors, item prefixes and per-descriptor status
// words, uploaded from pinned memory in one copy; the status words come back
// in a second copy; the event marks completion.
struct Iter {
    hipEvent_t ev = nullptr;
    uint8_t* h_buf = nullptr;   // pinned
    uint8_t* d_buf = nullptr;
    size_t cap = 0;
    bool busy = false;
    std::vector<uint64_t> members;    // tickets with chunks here, in descriptor order
    std::vector<bool> finishing;      // member's last chunk is here
    size_t status_off = 0;            // status words (one per member) in the buffers
};

struct Class {
    std::vector<DecDesc> descs;
    std::vector<uint64_t> prefix;
    std::vector<int> member;          // index into Iter::members
};

}  // namespace

struct zipnn_server_s {
    zipnn_ctx ctx = nullptr;
    zipnn_server_config cfg = {};
    hipStream_t stream = nullptr;
    uint8_t* pool = nullptr;
    std::map<uint64_t, uint64_t> free_;   // offset -> bytes, coalesced
    std::vector<Entry> entries;
    std::unordered_map<uint64_t, Req> reqs;
    std::deque<uint64_t> pending;         // submitted, waiting for admission
    std::vector<uint64_t> active;         // admitted, chunks left to launch (admission order)
    std::deque<uint64_t> done_q;          // completed, not yet handed out by next_done
    int admitted = 0;                     // admitted and not released
    Iter it[kIterDepth];
    int it_head = 0;                      // oldest iteration slot
    int it_busy = 0;
    uint64_t next_ticket = 1;
    zipnn_server_counters st = {};
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    bool stop = false;
    std::atomic<uint64_t> gen{0};         // bumped by submit, release and destroy
    std::thread th;
};

namespace {

bool pool_alloc(zipnn_server s, uint64_t bytes, uint64_t* off)
{
    for (auto itf = s->free_.begin(); itf != s->free_.end(); ++itf) {
        if (itf->second < bytes) continue;
        *off = itf->first;
        const uint64_t rest = itf->second - bytes, at = itf->first + bytes;
        s->free_.erase(itf);
        if (rest) s->free_[at] = rest;
        s->st.pool_in_use += bytes;
        s->st.pool_peak = std::max(s->st.pool_peak, s->st.pool_in_use);
        return true;
    }
    return false;
}

void pool_free(zipnn_server s, uint64_t off, uint64_t bytes)
{
    auto nx = s->free_.lower_bound(off);
    if (nx != s->free_.end() && off + bytes == nx->first) {
        bytes += nx->second;
        nx = s->free_.erase(nx);
    }
    if (nx != s->free_.begin()) {
        auto pv = std::prev(nx);
        if (pv->first + pv->second == off) {
            pv->second += bytes;
            return;
        }
    }
    s->free_[off] = bytes;
}

void finish(zipnn_server s, uint64_t ticket, Req& r, double t)
{
    r.state = kDone;
    r.t.t_done = t;
    s->st.completed++;
    s->st.bytes_out += r.bytes;
    s->done_q.push_back(ticket);
}

void admit(zipnn_server s)
{
    while (!s->pending.empty() && s->admitted < s->cfg.max_inflight) {
        const uint64_t ticket = s->pending.front();
        Req& r = s->reqs[ticket];
        uint64_t off = 0;
        const uint64_t held = round_up(std::max<uint64_t>(r.bytes, 1), kPoolAlign);
        if (!pool_alloc(s, held, &off)) break;   // in arrival order: the head waits for room
        s->pending.pop_front();
        r.off = off;
        r.held = held;
        r.state = kActive;
        r.t.t_admit = now_s();
        s->admitted++;
        s->st.active_peak = std::max(s->st.active_peak, s->admitted);
        if (r.n_chunks == 0) {
            r.t.t_launch = r.t.t_admit;
            finish(s, ticket, r, r.t.t_admit);
        } else {
            s->active.push_back(ticket);
        }
    }
}

bool grow_iter(Iter& it, size_t need)
{
    if (need <= it.cap) return true;
    size_t cap = std::max<size_t>(need, 64 << 10);
    uint8_t *h = nullptr, *d = nullptr;
    if (host_malloc((void**)&h, cap) != hipSuccess) return false;
    if (dev_malloc((void**)&d, cap) != hipSuccess) {
        (void)hipHostFree(h);
        return false;
    }
    if (it.h_buf) (void)hipHostFree(it.h_buf);
    if (it.d_buf) (void)hipFree(it.d_buf);
    it.h_buf = h;
    it.d_buf = d;
    it.cap = cap;
    return true;
}

// Take the next iteration's work from the admitted requests and queue it.
// Returns false if there was nothing to launch.
bool launch_iteration(zipnn_server s)
{
    if (s->active.empty() || s->it_busy == kIterDepth) return false;
    Iter& it = s->it[(s->it_head + s->it_busy) % kIterDepth];
    it.members.clear();
    it.finishing.clear();
    std::vector<std::pair<uint64_t, uint32_t>> take;   // ticket, chunks
    if (s->cfg.mode == ZIPNN_SERVE_PER_REQUEST) {
        const uint64_t ticket = s->active.front();
        const Req& r = s->reqs[ticket];
        take.push_back({ticket, r.n_chunks - r.next});
    } else {
        // whole requests: the oldest first (the largest requests set the
        // tail latency, and so they never wait behind later small ones),
        // then the others fewest chunks first while they fit under the
        // chunk cap.  At 5000 requests/s the p99 was 1.50 ms in this order,
        // 1.54 ms in arrival order and 1.81 ms with every request fewest
        // chunks first (older than 2 ms first); a burst of 128 requests had
        // its p50 at 1.6, 3.8 and 2.0 ms.  A request is never split: a split
        // only adds a launch to the largest requests, while those batched
        // with it would wait for the whole iteration anyway.
        // Batching only when requests would otherwise wait: while every
        // admitted request can have an iteration of its own in flight now,
        // each goes alone, as in per-request mode (a batch would hold its
        // oldest request until the others are decoded too).
        const size_t free_slots = size_t(kIterDepth - s->it_busy);
        const bool fill = s->active.size() > free_slots;
        std::vector<std::pair<uint32_t, uint64_t>> rest;   // chunks, ticket
        for (size_t i = 1; fill && i < s->active.size(); i++) {
            const Req& r = s->reqs[s->active[i]];
            rest.push_back({r.n_chunks - r.next, s->active[i]});
        }
        std::sort(rest.begin(), rest.end());
        const Req& r0 = s->reqs[s->active.front()];
        uint64_t used = r0.n_chunks - r0.next;
        take.push_back({s->active.front(), uint32_t(used)});
        for (auto& o : rest) {
            if (used + o.first > s->cfg.chunks_per_iter) continue;
            take.push_back({o.second, o.first});
            used += o.first;
        }
    }
    // descriptors by kernel class, in the order taken
    std::map<std::tuple<uint32_t, uint32_t, bool, bool>, Class> classes;
    const double t = now_s();
    for (auto& tk : take) {
        Req& r = s->reqs[tk.first];
        const Entry& e = s->entries[r.handle];
        DecDesc d;
        d.src = e.src;
        d.src_len = e.len;
        d.base = e.base;
        d.dst = s->pool + r.off;
        d.dst_cap = r.bytes;
        d.c_begin = r.next;
        d.c_end = r.next + tk.second;
        d.status = nullptr;   // set once the buffer layout is known
        const DecClass k = dec_class(e.h);
        Class& c = classes[std::make_tuple(k.B, k.G, k.delta, k.zg)];
        const uint64_t items = plan_items(e.h, d.c_begin, d.c_end).items;
        if (c.prefix.empty()) c.prefix.push_back(0);
        c.prefix.push_back(c.prefix.back() + items);
        c.descs.push_back(d);
        c.member.push_back(int(it.members.size()));
        it.members.push_back(tk.first);
        r.next += tk.second;
        it.finishing.push_back(r.next == r.n_chunks);
        if (!r.launched) {
            r.launched = true;
            r.t.t_launch = t;
        }
        s->st.chunks += tk.second;
    }
    // buffer layout: per class descriptors, then the item prefix and the
    // decode's item counter (zero), then the status words
    size_t off = 0;
    std::vector<std::pair<size_t, size_t>> at;   // per class: descs, prefix
    for (auto& kv : classes) {
        const size_t dd = off;
        off = round_up(off + kv.second.descs.size() * sizeof(DecDesc), 256);
        const size_t pp = off;
        off = round_up(off + (kv.second.prefix.size() + 1) * sizeof(uint64_t), 256);
        at.push_back({dd, pp});
    }
    it.status_off = off;
    const size_t total = off + it.members.size() * sizeof(int);
    int rc = grow_iter(it, total) ? ZIPNN_OK : ZIPNN_E_NOMEM;
    if (rc == ZIPNN_OK) {
        int* d_status = (int*)(it.d_buf + it.status_off);
        size_t ci = 0;
        for (auto& kv : classes) {
            Class& c = kv.second;
            for (size_t i = 0; i < c.descs.size(); i++) c.descs[i].status = d_status + c.member[i];
            memcpy(it.h_buf + at[ci].first, c.descs.data(), c.descs.size() * sizeof(DecDesc));
            memcpy(it.h_buf + at[ci].second, c.prefix.data(), c.prefix.size() * sizeof(uint64_t));
            memset(it.h_buf + at[ci].second + c.prefix.size() * sizeof(uint64_t), 0, sizeof(uint64_t));
            ci++;
        }
        memset(it.h_buf + it.status_off, 0, it.members.size() * sizeof(int));
        hipError_t e = hipMemcpyAsync(it.d_buf, it.h_buf, total, hipMemcpyHostToDevice, s->stream);
        ci = 0;
        for (auto& kv : classes) {
            if (e != hipSuccess) break;
            const Class& c = kv.second;
            const uint64_t items = c.prefix.back();
            const DecClass k{std::get<0>(kv.first), std::get<1>(kv.first), std::get<2>(kv.first),
                             std::get<3>(kv.first)};
            const int grid = int(std::min<uint64_t>(uint64_t(s->ctx->dec_grid[dec_class_index(k)]),
                                                    std::max<uint64_t>(items, 1)));
            e = launch_decode_planned(k, (const DecDesc*)(it.d_buf + at[ci].first), int(c.descs.size()),
                                      (uint64_t*)(it.d_buf + at[ci].second), d_status, grid, s->stream);
            ci++;
        }
        if (e == hipSuccess)
            e = hipMemcpyAsync(it.h_buf + it.status_off, it.d_buf + it.status_off, it.members.size() * sizeof(int),
                               hipMemcpyDeviceToHost, s->stream);
        if (e == hipSuccess) e = hipEventRecord(it.ev, s->stream);
        if (e != hipSuccess) rc = ZIPNN_E_HIP;
    }
    // drop fully launched requests from the active list
    s->active.erase(std::remove_if(s->active.begin(), s->active.end(),
                                   [&](uint64_t tk) {
                                       const Req& r = s->reqs[tk];
                                       return r.next == r.n_chunks;
                                   }),
                    s->active.end());
    s->st.iterations++;
    if (rc != ZIPNN_OK) {
        // nothing of this iteration is trusted: its members fail now
        const double td = now_s();
        for (size_t i = 0; i < it.members.size(); i++) {
            Req& r = s->reqs[it.members[i]];
            r.status = rc;
            if (it.finishing[i]) finish(s, it.members[i], r, td);
        }
        (void)hipStreamSynchronize(s->stream);
        s->cv_done.notify_all();
        return true;
    }
    it.busy = true;
    s->it_busy++;
    return true;
}

// Retire completed iterations, oldest first.  Returns how many retired.
int retire(zipnn_server s)
{
    int n = 0;
    while (s->it_busy > 0) {
        Iter& it = s->it[s->it_head];
        const hipError_t q = hipEventQuery(it.ev);
        if (q == hipErrorNotReady) break;
        const double t = now_s();
        const int* hs = (const int*)(it.h_buf + it.status_off);
        for (size_t i = 0; i < it.members.size(); i++) {
            Req& r = s->reqs[it.members[i]];
            const int code = q == hipSuccess ? hs[i] : ZIPNN_E_HIP;
            if (code != ZIPNN_OK && r.status == ZIPNN_OK) r.status = code;
            if (it.finishing[i]) finish(s, it.members[i], r, t);
        }
        it.busy = false;
        s->it_head = (s->it_head + 1) % kIterDepth;
        s->it_busy--;
        n++;
    }
    if (n) s->cv_done.notify_all();
    return n;
}

void scheduler(zipnn_server s)
{
    (void)hipSetDevice(s->ctx->device);
    for (;;) {
        uint64_t seen;
        hipEvent_t oldest = nullptr;
        {
            std::lock_guard<std::mutex> lk(s->mu);
            retire(s);
            if (!s->stop) {
                admit(s);
                while (launch_iteration(s)) {
                }
            }
            if (s->stop && s->it_busy == 0) break;
            seen = s->gen.load();
            if (s->it_busy > 0) oldest = s->it[s->it_head].ev;
        }
        // wait outside the lock, so that API calls are never held up: for the
        // oldest iteration in flight to complete or for a submit / release /
        // destroy; with nothing in flight, poll a while and then sleep
        if (oldest) {
            while (s->gen.load() == seen && hipEventQuery(oldest) == hipErrorNotReady) std::this_thread::yield();
        } else {
            const double t_spin = now_s() + kIdleSpinSeconds;
            while (s->gen.load() == seen && now_s() < t_spin) std::this_thread::yield();
            std::unique_lock<std::mutex> lk(s->mu);
            s->cv_work.wait(lk, [&] { return s->gen.load() != seen; });
        }
    }
}

}  // namespace

extern "C" {

double zipnn_clock(void) { return now_s(); }

int zipnn_server_create(zipnn_ctx ctx, const zipnn_server_config* cfg, zipnn_server* out)
{
    if (!out) return ZIPNN_E_INVAL;
    *out = nullptr;
    if (!ctx || !cfg || cfg->pool_bytes == 0 || cfg->max_inflight < 1 ||
        (cfg->mode != ZIPNN_SERVE_CONTINUOUS && cfg->mode != ZIPNN_SERVE_PER_REQUEST))
        return ZIPNN_E_INVAL;
    zipnn_server s = new (std::nothrow) zipnn_server_s;
    if (!s) return ZIPNN_E_NOMEM;
    s->ctx = ctx;
    s->cfg = *cfg;
    s->cfg.pool_bytes = round_up(cfg->pool_bytes, kPoolAlign);
    if (s->cfg.chunks_per_iter == 0) s->cfg.chunks_per_iter = kDefaultChunksPerIter;
    int prev = -1;
    (void)hipGetDevice(&prev);
    (void)hipSetDevice(ctx->device);
    int rc = ZIPNN_OK;
    if (dev_malloc((void**)&s->pool, s->cfg.pool_bytes) != hipSuccess) rc = ZIPNN_E_NOMEM;
    if (rc == ZIPNN_OK && hipStreamCreateWithFlags(&s->stream, hipStreamNonBlocking) != hipSuccess) rc = ZIPNN_E_HIP;
    for (int i = 0; rc == ZIPNN_OK && i < kIterDepth; i++) {
        if (hipEventCreateWithFlags(&s->it[i].ev, hipEventDisableTiming) != hipSuccess) rc = ZIPNN_E_HIP;
        else if (!grow_iter(s->it[i], size_t(s->cfg.max_inflight) * 96 + 4096)) rc = ZIPNN_E_NOMEM;
    }
    if (prev >= 0) (void)hipSetDevice(prev);
    if (rc != ZIPNN_OK) {
        zipnn_server_destroy(s);
        return rc;
    }
    s->free_[0] = s->cfg.pool_bytes;
    s->th = std::thread(scheduler, s);
    *out = s;
    return ZIPNN_OK;
}

void zipnn_server_destroy(zipnn_server s)
{
    if (!s) return;
    if (s->th.joinable()) {
        {
            std::lock_guard<std::mutex> lk(s->mu);
            s->stop = true;
            s->gen++;
        }
        s->cv_work.notify_all();
        s->th.join();
    }
    int prev = -1;
    (void)hipGetDevice(&prev);
    (void)hipSetDevice(s->ctx->device);
    if (s->stream) {
        (void)hipStreamSynchronize(s->stream);
        (void)hipStreamDestroy(s->stream);
    }
    for (auto& it : s->it) {
        if (it.ev) (void)hipEventDestroy(it.ev);
        if (it.h_buf) (void)hipHostFree(it.h_buf);
        if (it.d_buf) (void)hipFree(it.d_buf);
    }
    if (s->pool) (void)hipFree(s->pool);
    if (prev >= 0) (void)hipSetDevice(prev);
    delete s;
}

int zipnn_server_register(zipnn_server s, const void* src, uint64_t src_len, const void* base, uint32_t* handle)
{
    if (!s || !src || !handle || src_len < 64 || (reinterpret_cast<uintptr_t>(src) & 15u) ||
        (reinterpret_cast<uintptr_t>(base) & 15u))
        return ZIPNN_E_INVAL;
    uint32_t w[16];
    int prev = -1;
    (void)hipGetDevice(&prev);
    (void)hipSetDevice(s->ctx->device);
    const hipError_t e = hipMemcpy(w, src, 64, hipMemcpyDeviceToHost);
    if (prev >= 0) (void)hipSetDevice(prev);
    if (e != hipSuccess) return ZIPNN_E_HIP;
    Entry en;
    const int rc = parse_header(w, src_len, en.h);
    if (rc != ZIPNN_OK) return rc;
    if (((en.h.flags & kFlagDelta) != 0) != (base != nullptr)) return ZIPNN_E_INVAL;
    en.src = (const uint8_t*)src;
    en.len = src_len;
    en.base = (const uint8_t*)base;
    std::lock_guard<std::mutex> lk(s->mu);
    *handle = uint32_t(s->entries.size());
    s->entries.push_back(en);
    return ZIPNN_OK;
}

int zipnn_server_submit(zipnn_server s, uint32_t handle, double t_arrive, uint64_t* ticket)
{
    if (!s || !ticket) return ZIPNN_E_INVAL;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        if (handle >= s->entries.size()) return ZIPNN_E_INVAL;
        const Header& h = s->entries[handle].h;
        Req r;
        r.handle = handle;
        r.bytes = h.n * h.B;
        r.n_chunks = h.n_chunks;
        if (round_up(std::max<uint64_t>(r.bytes, 1), kPoolAlign) > s->cfg.pool_bytes) return ZIPNN_E_NOSPACE;
        r.t.t_arrive = t_arrive > 0 ? t_arrive : now_s();
        const uint64_t tk = s->next_ticket++;
        s->reqs.emplace(tk, r);
        s->pending.push_back(tk);
        s->st.submitted++;
        s->gen++;
        *ticket = tk;
    }
    s->cv_work.notify_one();
    return ZIPNN_OK;
}

int zipnn_server_poll(zipnn_server s, uint64_t ticket, void** out, zipnn_timing* t)
{
    if (!s) return ZIPNN_E_INVAL;
    std::lock_guard<std::mutex> lk(s->mu);
    auto f = s->reqs.find(ticket);
    if (f == s->reqs.end()) return ZIPNN_E_INVAL;
    const Req& r = f->second;
    if (r.state != kDone) return ZIPNN_E_BUSY;
    if (out) *out = s->pool + r.off;
    if (t) *t = r.t;
    return r.status;
}

int zipnn_server_next_done(zipnn_server s, double timeout_s, uint64_t* ticket)
{
    if (!s || !ticket) return ZIPNN_E_INVAL;
    std::unique_lock<std::mutex> lk(s->mu);
    const auto until = std::chrono::steady_clock::now() +
                       std::chrono::nanoseconds(int64_t(std::max(0.0, timeout_s) * 1e9));
    for (;;) {
        while (!s->done_q.empty()) {
            const uint64_t tk = s->done_q.front();
            s->done_q.pop_front();
            if (s->reqs.count(tk)) {
                *ticket = tk;
                return ZIPNN_OK;
            }
        }
        if (s->cv_done.wait_until(lk, until) == std::cv_status::timeout && s->done_q.empty()) return ZIPNN_E_BUSY;
    }
}

int zipnn_server_release(zipnn_server s, uint64_t ticket)
{
    if (!s) return ZIPNN_E_INVAL;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        auto f = s->reqs.find(ticket);
        if (f == s->reqs.end()) return ZIPNN_E_INVAL;
        if (f->second.state != kDone) return ZIPNN_E_BUSY;
        pool_free(s, f->second.off, f->second.held);
        s->st.pool_in_use -= f->second.held;
        s->admitted--;
        s->st.released++;
        s->gen++;
        s->reqs.erase(f);
    }
    s->cv_work.notify_one();
    return ZIPNN_OK;
}

int zipnn_server_stats(zipnn_server s, zipnn_server_counters* out)
{
    if (!s || !out) return ZIPNN_E_INVAL;
    std::lock_guard<std::mutex> lk(s->mu);
    *out = s->st;
    return ZIPNN_OK;
}

int zipnn_server_set_mode(zipnn_server s, int mode)
{
    if (!s || (mode != ZIPNN_SERVE_CONTINUOUS && mode != ZIPNN_SERVE_PER_REQUEST)) return ZIPNN_E_INVAL;
    std::lock_guard<std::mutex> lk(s->mu);   // launch_iteration reads the mode under this lock
    s->cfg.mode = mode;
    return ZIPNN_OK;
}

}  // extern "C"
