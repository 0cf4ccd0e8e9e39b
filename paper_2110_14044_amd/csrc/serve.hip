// Fold-in server: continuous batching of new-row fold-ins against a resident
// item table (the fold-in of foldin.hip, one workgroup per request).
//
// Admission.  A request is admitted when a slot is free and the device arena
// (the HBM budget) has a contiguous region for its state: the prediction cache,
// staged ids and labels (and the factors when they do not fit in LDS).  The
// pinned host arena mirrors the device arena offset for offset: the submitting
// thread copies the ids and labels into the host side of the region, the
// kernel stages them into the device side, and writes the result row and a
// status word back into the host side.  A request therefore costs no copy
// call of its own, and a batch is one kernel launch plus one event.
//
// Batching.  A worker thread owns `streams` streams.  Whenever one of them is
// free and requests are waiting, everything admitted so far becomes one batch
// on that stream, while the batches on the other streams keep running; a
// stream becomes free when the event recorded after its batch has completed.
// Results wait in the done queue until ials_server_poll copies them out and
// frees their slot and region.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <climits>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <thread>
#include <vector>

#include "ials_internal.h"

namespace {

thread_local std::string g_server_create_error;

// First-fit allocator over [0, cap) in 256-byte granules, merging neighbours on release.
class Arena {
  public:
    static constexpr size_t npos = SIZE_MAX;
    void reset(size_t cap) {
        cap_ = cap;
        used_ = 0;
        free_.clear();
        if (cap) free_[0] = cap;
    }
    static size_t granule(size_t bytes) { return (bytes + 255) / 256 * 256; }
    size_t alloc(size_t bytes) {
        bytes = granule(bytes);
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second < bytes) continue;
            const size_t off = it->first, sz = it->second;
            free_.erase(it);
            if (sz > bytes) free_[off + bytes] = sz - bytes;
            used_ += bytes;
            return off;
        }
        return npos;
    }
    void release(size_t off, size_t bytes) {
        bytes = granule(bytes);
        used_ -= bytes;
        auto it = free_.emplace(off, bytes).first;
        auto nx = std::next(it);
        if (nx != free_.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free_.erase(nx);
        }
        if (it != free_.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_.erase(it);
            }
        }
    }
    size_t used() const { return used_; }
    size_t capacity() const { return cap_; }

  private:
    size_t cap_ = 0, used_ = 0;
    std::map<size_t, size_t> free_;
};

struct Req {
    uint64_t tag = 0;
    size_t off = 0, bytes = 0;
    int32_t n = 0;
    bool has_y = false;
};

struct Batch {
    std::vector<Req> reqs;
    bool active = false;
};

}  // namespace

struct ials_server {
    ials::FoldShape fold;
    int device = 0;
    float alpha0 = 0.f, lambda = 0.f, tau = 1e-4f;
    int32_t passes = 0, max_slots = 1, nstreams = 4;
    const float* H = nullptr;
    float* G = nullptr;
    int32_t* cnt = nullptr;
    char* dev_arena = nullptr;
    char* host_arena = nullptr;  // pinned, host view
    char* host_arena_dev = nullptr;  // the same memory as the device addresses it
    Arena arena;
    std::vector<hipStream_t> streams;
    std::vector<hipEvent_t> events;
    std::vector<ials::FoldReq*> desc;      // pinned, host view, max_slots per stream
    std::vector<ials::FoldReq*> desc_dev;  // device view
    std::vector<Batch> batches;

    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<Req> pending, done;
    int32_t admitted = 0;
    bool stop = false;
    std::string fatal;
    std::thread worker;
    ials_server_stats st{};
    std::string err;

    size_t out_off(int32_t n) const { return ials::fold_ws_floats(fold, n) * sizeof(float); }
    size_t region_bytes(int32_t n) const {
        return out_off(n) + (size_t)(fold.d + 1 + 63) / 64 * 64 * sizeof(float);
    }
};

namespace {

void fill_desc(ials_server* s, const Req& q, ials::FoldReq& d) {
    const size_t n = (size_t)q.n;
    float* hbase = reinterpret_cast<float*>(s->host_arena_dev + q.off);
    d.items = reinterpret_cast<const int32_t*>(hbase + 2 * n);
    d.y = q.has_y ? hbase + 3 * n : nullptr;
    d.ws = reinterpret_cast<float*>(s->dev_arena + q.off);
    d.out = reinterpret_cast<float*>(s->host_arena_dev + q.off + s->out_off(q.n));
    d.st = reinterpret_cast<int32_t*>(d.out + s->fold.d);
    d.n = q.n;
    d.copy = 1;
}

void worker_main(ials_server* s) {
    (void)hipSetDevice(s->device);
    std::unique_lock<std::mutex> lk(s->mu);
    for (;;) {
        // finished batches move to the done queue
        bool running = false;
        for (int q = 0; q < s->nstreams; ++q) {
            Batch& b = s->batches[q];
            if (!b.active) continue;
            const hipError_t e = hipEventQuery(s->events[q]);
            if (e == hipErrorNotReady) {
                running = true;
                continue;
            }
            if (e != hipSuccess && s->fatal.empty())
                s->fatal = std::string("fold-in batch failed: ") + hipGetErrorString(e);
            if (e == hipSuccess) {
                for (const Req& r : b.reqs) s->done.push_back(r);
                s->st.completed += (int64_t)b.reqs.size();
            } else {
                for (const Req& r : b.reqs) s->arena.release(r.off, r.bytes);
                s->admitted -= (int32_t)b.reqs.size();
            }
            b.reqs.clear();
            b.active = false;
            s->st.in_flight -= 1;
            s->cv_done.notify_all();
        }
        if (s->stop) {
            for (const Req& r : s->pending) s->arena.release(r.off, r.bytes);
            s->admitted -= (int32_t)s->pending.size();
            s->pending.clear();
            if (!running) break;
        }
        // everything admitted so far goes out on the first free stream
        int freeq = -1;
        for (int q = 0; q < s->nstreams && freeq < 0; ++q)
            if (!s->batches[q].active) freeq = q;
        if (freeq >= 0 && !s->pending.empty() && s->fatal.empty()) {
            Batch& b = s->batches[freeq];
            const size_t m = std::min(s->pending.size(), (size_t)s->max_slots);
            b.reqs.assign(s->pending.begin(), s->pending.begin() + (std::ptrdiff_t)m);
            s->pending.erase(s->pending.begin(), s->pending.begin() + (std::ptrdiff_t)m);
            b.active = true;
            s->st.batches += 1;
            s->st.max_batch = std::max<int64_t>(s->st.max_batch, (int64_t)m);
            s->st.in_flight += 1;
            lk.unlock();
            for (size_t i = 0; i < m; ++i) fill_desc(s, b.reqs[i], s->desc[freeq][i]);
            hipError_t e = ials::launch_foldin(s->streams[freeq], s->fold, s->H, s->G, s->alpha0, s->lambda, s->tau,
                                               s->passes, s->desc_dev[freeq], (int32_t)m, s->cnt);
            if (e == hipSuccess) e = hipEventRecord(s->events[freeq], s->streams[freeq]);
            lk.lock();
            if (e != hipSuccess && s->fatal.empty())
                s->fatal = std::string("fold-in launch failed: ") + hipGetErrorString(e);
            continue;
        }
        if (!running) {
            s->cv_work.wait(lk, [s] { return s->stop || (!s->pending.empty() && s->fatal.empty()); });
        } else {
            lk.unlock();
            std::this_thread::yield();
            lk.lock();
        }
    }
}

void free_server(ials_server* s) {
    if (!s) return;
    if (s->worker.joinable()) {
        {
            std::lock_guard<std::mutex> g(s->mu);
            s->stop = true;
        }
        s->cv_work.notify_all();
        s->worker.join();
    }
    for (hipStream_t q : s->streams)
        if (q) (void)hipStreamSynchronize(q);
    for (hipEvent_t e : s->events)
        if (e) (void)hipEventDestroy(e);
    for (hipStream_t q : s->streams)
        if (q) (void)hipStreamDestroy(q);
    for (ials::FoldReq* p : s->desc)
        if (p) (void)hipHostFree(p);
    if (s->host_arena) (void)hipHostFree(s->host_arena);
    if (s->dev_arena) (void)hipFree(s->dev_arena);
    if (s->G) (void)hipFree(s->G);
    if (s->cnt) (void)hipFree(s->cnt);
    delete s;
}

#define SRV_TRY(expr)                                                                    \
    do {                                                                                 \
        hipError_t e_ = (expr);                                                          \
        if (e_ != hipSuccess) {                                                          \
            g_server_create_error = std::string(#expr " failed: ") + hipGetErrorString(e_); \
            free_server(s);                                                              \
            return IALS_E_HIP;                                                           \
        }                                                                                \
    } while (0)

ials_status create_server(const ials_server_config* cfg, const float* H, ials_server** out) {
    if (!cfg || !H || !out) {
        g_server_create_error = "null argument";
        return IALS_E_INVALID;
    }
    *out = nullptr;
    if (cfg->num_items < 1 || cfg->dim < 1 || cfg->block < 1 || cfg->block > cfg->dim || cfg->block > 64) {
        g_server_create_error = "need num_items >= 1, dim >= 1 and 1 <= block <= min(dim, 64)";
        return IALS_E_INVALID;
    }
    if (!(cfg->alpha0 >= 0.f) || !(cfg->lambda > 0.f) || !std::isfinite(cfg->alpha0) || !std::isfinite(cfg->lambda)) {
        g_server_create_error = "need alpha0 >= 0 and lambda > 0 (finite)";
        return IALS_E_INVALID;
    }
    if (cfg->precision != IALS_PREC_FP32) {
        g_server_create_error = "only IALS_PREC_FP32 is available for serving";
        return IALS_E_INVALID;
    }
    if (cfg->passes < 0 || cfg->passes > 1000 || cfg->max_slots < 1 || cfg->max_slots > (1 << 20) ||
        cfg->streams < 0 || cfg->streams > 8) {
        g_server_create_error = "need 0 <= passes <= 1000, 1 <= max_slots <= 2^20 and 0 <= streams <= 8";
        return IALS_E_INVALID;
    }
    const uint64_t budget = cfg->hbm_budget ? cfg->hbm_budget : ((uint64_t)64 << 20);
    if (budget < ((uint64_t)1 << 20) || budget > ((uint64_t)64 << 30)) {
        g_server_create_error = "hbm_budget must be between 1 MiB and 64 GiB";
        return IALS_E_INVALID;
    }
    ials::FoldShape f = ials::fold_shape(cfg->num_items, cfg->dim, cfg->block);
    ials_server* s = new (std::nothrow) ials_server();
    if (!s) {
        g_server_create_error = "host allocation failed";
        return IALS_E_NOMEM;
    }
    s->fold = f;
    s->alpha0 = cfg->alpha0;
    s->lambda = cfg->lambda;
    s->tau = ials::effective_tau(cfg->chol_fallback_ratio);
    s->passes = cfg->passes;
    s->max_slots = cfg->max_slots;
    s->nstreams = cfg->streams ? cfg->streams : 4;
    s->H = H;
    SRV_TRY(hipGetDevice(&s->device));
    s->streams.assign(s->nstreams, nullptr);
    s->events.assign(s->nstreams, nullptr);
    s->desc.assign(s->nstreams, nullptr);
    s->desc_dev.assign(s->nstreams, nullptr);
    s->batches.resize(s->nstreams);
    for (int q = 0; q < s->nstreams; ++q) {
        SRV_TRY(hipStreamCreateWithFlags(&s->streams[q], hipStreamNonBlocking));
        SRV_TRY(hipEventCreateWithFlags(&s->events[q], hipEventDisableTiming));
        void* p = nullptr;
        SRV_TRY(hipHostMalloc(&p, sizeof(ials::FoldReq) * s->max_slots, hipHostMallocMapped));
        s->desc[q] = static_cast<ials::FoldReq*>(p);
        void* pd = nullptr;
        SRV_TRY(hipHostGetDevicePointer(&pd, p, 0));
        s->desc_dev[q] = static_cast<ials::FoldReq*>(pd);
    }
    const size_t dd = (size_t)f.d * f.d;
    SRV_TRY(hipMalloc((void**)&s->G, sizeof(float) * dd));
    SRV_TRY(hipMalloc((void**)&s->cnt, sizeof(int32_t) * ials::FOLD_CNT_NUM));
    SRV_TRY(hipMemsetAsync(s->cnt, 0, sizeof(int32_t) * ials::FOLD_CNT_NUM, s->streams[0]));
    {
        float* part = nullptr;
        SRV_TRY(hipMalloc((void**)&part, sizeof(float) * ials::gram_part_floats_needed(f.I, f.d, f.d, false)));
        ials::launch_gramian_raw(s->streams[0], H, f.I, f.d, 0, f.d, f.d, part, s->G, false);
        hipError_t e = hipGetLastError();
        if (e == hipSuccess) e = hipStreamSynchronize(s->streams[0]);
        (void)hipFree(part);
        SRV_TRY(e);
    }
    SRV_TRY(hipMalloc((void**)&s->dev_arena, budget));
    {
        void* p = nullptr;
        SRV_TRY(hipHostMalloc(&p, budget, hipHostMallocMapped | hipHostMallocCoherent));
        s->host_arena = static_cast<char*>(p);
        void* pd = nullptr;
        SRV_TRY(hipHostGetDevicePointer(&pd, p, 0));
        s->host_arena_dev = static_cast<char*>(pd);
    }
    s->arena.reset(budget);
    s->st.arena_bytes = budget;
    try {
        s->worker = std::thread(worker_main, s);
    } catch (...) {
        g_server_create_error = "could not start the worker thread";
        free_server(s);
        return IALS_E_NOMEM;
    }
    *out = s;
    return IALS_OK;
}

}  // namespace

extern "C" {

ials_status ials_server_create(const ials_server_config* cfg, const float* H, ials_server** out) {
    try {
        g_server_create_error.clear();
        return create_server(cfg, H, out);
    } catch (...) {
        g_server_create_error = "unexpected host exception in ials_server_create";
        return IALS_E_NOMEM;
    }
}

ials_status ials_server_submit(ials_server* s, int32_t n, const int32_t* items, const float* y, uint64_t tag) {
    if (!s) return IALS_E_INVALID;
    try {
        if (n < 0 || (n > 0 && !items)) {
            std::lock_guard<std::mutex> g(s->mu);
            s->err = "need n >= 0 and non-null items";
            return IALS_E_INVALID;
        }
        for (int32_t k = 0; k < n; ++k)
            if ((unsigned)items[k] >= (unsigned)s->fold.I) {
                std::lock_guard<std::mutex> g(s->mu);
                s->err = "item id out of range at position " + std::to_string(k);
                return IALS_E_INVALID;
            }
        const size_t bytes = s->region_bytes(n);
        Req q;
        {
            std::lock_guard<std::mutex> g(s->mu);
            if (bytes > s->arena.capacity()) {
                s->err = "request needs " + std::to_string(bytes) + " arena bytes, more than hbm_budget";
                return IALS_E_INVALID;
            }
            if (!s->fatal.empty() || s->stop) {
                s->err = s->fatal.empty() ? "server is stopping" : s->fatal;
                return IALS_E_STATE;
            }
            if (s->admitted >= s->max_slots) {
                s->st.rejected_busy += 1;
                return IALS_E_BUSY;
            }
            const size_t off = s->arena.alloc(bytes);
            if (off == Arena::npos) {
                s->st.rejected_busy += 1;
                return IALS_E_BUSY;
            }
            s->admitted += 1;
            s->st.bytes_peak = std::max<uint64_t>(s->st.bytes_peak, s->arena.used());
            q.tag = tag;
            q.off = off;
            q.bytes = bytes;
            q.n = n;
            q.has_y = y != nullptr;
        }
        // the region is ours: stage the inputs in its host half without the lock
        float* hbase = reinterpret_cast<float*>(s->host_arena + q.off);
        if (n > 0) std::memcpy(hbase + 2 * (size_t)n, items, sizeof(int32_t) * (size_t)n);
        if (y && n > 0) std::memcpy(hbase + 3 * (size_t)n, y, sizeof(float) * (size_t)n);
        {
            std::lock_guard<std::mutex> g(s->mu);
            s->pending.push_back(q);
            s->st.submitted += 1;
        }
        s->cv_work.notify_one();
        return IALS_OK;
    } catch (...) {
        return IALS_E_NOMEM;
    }
}

ials_status ials_server_poll(ials_server* s, int32_t max, int32_t wait_us, uint64_t* tags, float* w_out,
                             int32_t* status, int32_t* n_done) {
    if (!s || !n_done || max < 0 || (max > 0 && (!tags || !w_out))) return IALS_E_INVALID;
    *n_done = 0;
    try {
        std::unique_lock<std::mutex> lk(s->mu);
        if (s->done.empty() && wait_us > 0 && max > 0)
            s->cv_done.wait_for(lk, std::chrono::microseconds(wait_us),
                                [s] { return !s->done.empty() || !s->fatal.empty(); });
        const int32_t d = s->fold.d;
        int32_t k = 0;
        while (k < max && !s->done.empty()) {
            const Req q = s->done.front();
            s->done.pop_front();
            const float* o = reinterpret_cast<const float*>(s->host_arena + q.off + s->out_off(q.n));
            std::memcpy(w_out + (size_t)k * d, o, sizeof(float) * d);
            int32_t stw = 0;
            std::memcpy(&stw, o + d, sizeof(int32_t));
            const int32_t code = (stw & ials::FOLD_ST_NOT_SPD) ? 2 : ((stw & ials::FOLD_ST_FLOAT64) ? 1 : 0);
            if (status) status[k] = code;
            if (stw & ials::FOLD_ST_FLOAT64) s->st.float64_requests += 1;
            if (stw & ials::FOLD_ST_NOT_SPD) s->st.not_spd_requests += 1;
            tags[k] = q.tag;
            s->arena.release(q.off, q.bytes);
            s->admitted -= 1;
            s->st.polled += 1;
            ++k;
        }
        *n_done = k;
        if (!s->fatal.empty()) {
            s->err = s->fatal;
            return IALS_E_HIP;
        }
        return IALS_OK;
    } catch (...) {
        return IALS_E_NOMEM;
    }
}

ials_status ials_server_stats_get(ials_server* s, ials_server_stats* out) {
    if (!s || !out) return IALS_E_INVALID;
    std::lock_guard<std::mutex> g(s->mu);
    *out = s->st;
    out->admitted = s->admitted;
    out->bytes_in_use = s->arena.used();
    return IALS_OK;
}

ials_status ials_server_destroy(ials_server* s) {
    if (!s) return IALS_E_INVALID;
    free_server(s);
    return IALS_OK;
}

const char* ials_server_last_error(const ials_server* s) {
    if (!s) return g_server_create_error.c_str();
    return s->err.c_str();
}

}  // extern "C"
