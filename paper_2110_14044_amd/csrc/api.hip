// C-ABI entry points of libials: context lifecycle and the drivers of Alg. 3.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "ials_internal.h"

namespace {
thread_local std::string g_create_error;

void free_ctx(ials_ctx* c) {
    if (!c) return;
    (void)hipStreamSynchronize(c->stream);
    if (c->epoch_exec) (void)hipGraphExecDestroy(c->epoch_exec);
    for (void* p : c->owned) (void)hipFree(p);
    for (void* p : c->owned_host) (void)hipHostFree(p);
    for (hipEvent_t e : c->prof_pool) (void)hipEventDestroy(e);
    if (c->own_stream) (void)hipStreamDestroy(c->stream);
    delete c;
}

struct CreateGuard {
    ials_ctx* c;
    bool armed = true;
    ~CreateGuard() {
        if (armed && c) free_ctx(c);
    }
};

}  // namespace

namespace ials {

int resident_per_cu(OccCache& cache, const void* kernel, int threads, size_t lds, bool set_lds, int fallback) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= OccCache::kDevices) return fallback;
    int nb = cache.v[dev].load(std::memory_order_relaxed);
    if (nb > 0) return nb;
    if (set_lds && hipFuncSetAttribute(kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) != hipSuccess)
        return fallback;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, kernel, threads, lds) != hipSuccess || nb < 1) nb = fallback;
    cache.v[dev].store(nb, std::memory_order_relaxed);
    return nb;
}

hipError_t dev_alloc(ials_ctx* c, void** p, size_t bytes) {
    *p = nullptr;
    if (bytes == 0) bytes = 16;
    if (c->budget && c->device_bytes + c->tmp_bytes + bytes > c->budget) return hipErrorOutOfMemory;
    hipError_t e = hipMalloc(p, bytes);
    if (e != hipSuccess) {
        *p = nullptr;
        return e;
    }
    c->owned.push_back(*p);
    c->device_bytes += bytes;
    c->peak_bytes = std::max(c->peak_bytes, c->device_bytes + c->tmp_bytes);
    return hipSuccess;
}

hipError_t tmp_alloc(ials_ctx* c, void** p, size_t bytes) {
    *p = nullptr;
    if (bytes == 0) bytes = 16;
    if (c->budget && c->device_bytes + c->tmp_bytes + bytes > c->budget) return hipErrorOutOfMemory;
    hipError_t e = hipMalloc(p, bytes);
    if (e != hipSuccess) {
        *p = nullptr;
        return e;
    }
    c->tmp_bytes += bytes;
    c->peak_bytes = std::max(c->peak_bytes, c->device_bytes + c->tmp_bytes);
    return hipSuccess;
}

void tmp_free(ials_ctx* c, void* p, size_t bytes) {
    if (!p) return;
    (void)hipFree(p);
    c->tmp_bytes -= bytes == 0 ? 16 : bytes;
}

}  // namespace ials

namespace {

ials_status fail(ials_ctx* c, ials_status s, const std::string& msg) {
    if (c)
        c->err = msg;
    else
        g_create_error = msg;
    return s;
}

#define TRY_ALLOC(c, ptr, bytes)                                                           \
    do {                                                                                   \
        hipError_t e_ = ials::dev_alloc((c), (void**)&(ptr), (bytes));                     \
        if (e_ != hipSuccess) {                                                            \
            g_create_error = std::string("device allocation of ") + std::to_string(bytes) + \
                             " bytes failed (" + hipGetErrorString(e_) + ")";              \
            if ((c)->budget && e_ == hipErrorOutOfMemory)                                  \
                g_create_error += ": the HBM budget of " + std::to_string((c)->budget) +   \
                                  " bytes would be exceeded";                              \
            return ials::alloc_status(e_);                                                 \
        }                                                                                  \
    } while (0)

#define TRY_HIP_CREATE(expr)                                                               \
    do {                                                                                   \
        hipError_t e_ = (expr);                                                            \
        if (e_ != hipSuccess) {                                                            \
            g_create_error = std::string(#expr " failed: ") + hipGetErrorString(e_);      \
            return IALS_E_HIP;                                                             \
        }                                                                                  \
    } while (0)

ials_status check_ctx(ials_ctx* c) {
    if (!c) {
        g_create_error = "null context";
        return IALS_E_INVALID;
    }
    return IALS_OK;
}

int32_t block_width(const ials_ctx* c, int32_t blk) {
    const int32_t p0 = blk * c->b;
    return std::min(c->b, c->d - p0);
}

// The solver a block size selects: b = d is Alg. 1 (each row solved exactly against the
// dense normal equations, eq. 3), b = 1 is Alg. 2 (scalar coordinate descent), anything in
// between the block steps of Alg. 3.
int32_t solver_of(const ials_ctx* c) {
    if (c->b == 1) return IALS_SOLVER_ICD;
    if (c->b == c->d) return IALS_SOLVER_IALS;
    return IALS_SOLVER_BLOCK;
}

ials_status run_pass(ials_ctx* c, int side, int32_t blk) {
    const int32_t p0 = blk * c->b;
    const int32_t bw = block_width(c, blk);
    const bool user = side == IALS_SIDE_USER;
    const float* Xo = user ? c->H : c->W;
    const int32_t no = user ? c->I : c->U;
    float* X = user ? c->W : c->H;
    const int32_t n = user ? c->U : c->I;
    const int32_t solver = solver_of(c);
    if (solver == IALS_SOLVER_ICD) {
        // Alg. 2: the Gramian column, the dense term and the step are inside the iCD pass
        ials::launch_sweep(c, side, blk);
        c->passes += 1;
        IALS_HIP_TRY(c, hipGetLastError());
        return IALS_OK;
    }
    {
        ials::ProfScope ps(c, IALS_K_GRAM_USER + side);
        ials::launch_gramian_slab(c, Xo, no, p0, bw, c->B, c->G, true);
    }
    {
        ials::ProfScope ps(c, IALS_K_DENSE_USER + side);
        if (solver == IALS_SOLVER_IALS) {
            // Alg. 1: w = (alpha0 G + lambda I + sum alpha h h^T)^-1 sum alpha y h.  The row pass
            // computes it as its Newton step from w = 0 with no dense term: the residual of every
            // observation is then -y (the prediction cache is 0 when the block spans d), so the
            // gradient is -sum alpha y h and the new row is 0 - delta.
            ials::launch_fill(c->stream, X, (int64_t)n * c->d, 0.f);
            ials::launch_fill(c->stream, c->R0, (int64_t)n * c->B, 0.f);
        } else {
            ials::launch_dense(c, X, n, p0, bw);
        }
    }
    ials::launch_sweep(c, side, blk);
    c->passes += 1;
    IALS_HIP_TRY(c, hipGetLastError());
    return IALS_OK;
}

ials_status create_impl(const ials_config* cfg, const ials_coo* S, float* W, float* H, void* stream,
                        ials_ctx** out) {
    if (!cfg || !S || !W || !H || !out) {
        g_create_error = "null argument";
        return IALS_E_INVALID;
    }
    *out = nullptr;
    if (cfg->num_users < 1 || cfg->num_items < 1 || cfg->dim < 1 || cfg->block < 1 || cfg->block > cfg->dim ||
        cfg->block > 256) {
        g_create_error = "need num_users >= 1, num_items >= 1, dim >= 1 and 1 <= block <= min(dim, 256)";
        return IALS_E_INVALID;
    }
    if (!(cfg->alpha0 >= 0.f) || !(cfg->lambda > 0.f) || !std::isfinite(cfg->alpha0) || !std::isfinite(cfg->lambda)) {
        g_create_error = "need alpha0 >= 0 and lambda > 0 (finite)";
        return IALS_E_INVALID;
    }
    if (cfg->precision != IALS_PREC_FP32 && cfg->precision != IALS_PREC_BF16) {
        g_create_error = "precision must be IALS_PREC_FP32 or IALS_PREC_BF16";
        return IALS_E_INVALID;
    }
    if ((cfg->flags & ~(uint32_t)(IALS_FLAG_GRAPH | IALS_FLAG_DEAL_QUEUE | IALS_FLAG_DEAL_STATIC)) != 0 ||
        ((cfg->flags & IALS_FLAG_DEAL_QUEUE) && (cfg->flags & IALS_FLAG_DEAL_STATIC))) {
        g_create_error = "unknown or conflicting flag bits";
        return IALS_E_INVALID;
    }
    if (cfg->gram_split != 0 && (cfg->gram_split < 64 || cfg->gram_split > 2048 ||
                                 (cfg->gram_split & (cfg->gram_split - 1)) != 0)) {
        g_create_error = "gram_split must be 0 or a power of two in [64, 2048]";
        return IALS_E_INVALID;
    }
    if (cfg->seg_len != 0 && (cfg->seg_len % 64 != 0 || cfg->seg_len < 256 || cfg->seg_len > 65536)) {
        g_create_error = "seg_len must be 0 or a multiple of 64 in [256, 65536]";
        return IALS_E_INVALID;
    }
    if (S->nnz < 0 || S->nnz > (int64_t)INT32_MAX || (S->nnz > 0 && (!S->user || !S->item)) ||
        (S->memkind != IALS_MEM_HOST && S->memkind != IALS_MEM_DEVICE)) {
        g_create_error = "bad observation set (nnz must be in [0, 2^31), arrays non-null, memkind host or device)";
        return IALS_E_INVALID;
    }
    if ((int64_t)cfg->num_users * cfg->dim > ((int64_t)1 << 40) ||
        (int64_t)cfg->num_items * cfg->dim > ((int64_t)1 << 40)) {
        g_create_error = "embedding tables too large";
        return IALS_E_INVALID;
    }

    ials_ctx* c = new (std::nothrow) ials_ctx();
    if (!c) {
        g_create_error = "host allocation failed";
        return IALS_E_NOMEM;
    }
    CreateGuard guard{c};
    c->U = cfg->num_users;
    c->I = cfg->num_items;
    c->d = cfg->dim;
    c->b = cfg->block;
    // padded block: a multiple of 16 up to 64; 128 or 256 for the wide-block kernels
    c->B = cfg->block <= 64 ? (cfg->block + 15) / 16 * 16 : (cfg->block <= 128 ? 128 : 256);
    c->alpha0 = cfg->alpha0;
    c->lambda = cfg->lambda;
    c->tau = ials::effective_tau(cfg->chol_fallback_ratio);
    c->precision = cfg->precision;
    c->seg_len = cfg->seg_len ? (int32_t)cfg->seg_len : ials::kSegLenDefault;
    c->gram_split = cfg->gram_split ? (int32_t)cfg->gram_split : ials::kGramSplitDefault;
    c->nnz = S->nnz;
    c->stream = (hipStream_t)stream;
    c->W = W;
    c->H = H;
    c->budget = cfg->hbm_budget;
    c->flags = cfg->flags;
    if ((c->flags & IALS_FLAG_GRAPH) && c->stream == nullptr) {
        TRY_HIP_CREATE(hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking));
        c->own_stream = true;
    }
    TRY_HIP_CREATE(hipGetDevice(&c->device));
    int ncu = 0;
    TRY_HIP_CREATE(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, c->device));
    c->num_cu = std::max(ncu, 1);

    const int64_t nnz = c->nnz;
    const bool has_y = S->y != nullptr, has_a = S->alpha != nullptr;
    ials::SideIndex& us = c->side[IALS_SIDE_USER];
    ials::SideIndex& is = c->side[IALS_SIDE_ITEM];
    us.nrows = c->U;
    is.nrows = c->I;
    TRY_ALLOC(c, c->counters, sizeof(unsigned long long) * ials::CNT_NUM);
    TRY_ALLOC(c, c->cursors, sizeof(int32_t) * ials::CUR_NUM);
    TRY_HIP_CREATE(hipMemsetAsync(c->counters, 0, sizeof(unsigned long long) * ials::CNT_NUM, c->stream));
    TRY_HIP_CREATE(hipMemsetAsync(c->cursors, 0, sizeof(int32_t) * ials::CUR_NUM, c->stream));
    for (int sd = 0; sd < 2; ++sd) {
        ials::SideIndex& s = c->side[sd];
        TRY_ALLOC(c, s.ptr, sizeof(int64_t) * (s.nrows + 1));
        TRY_ALLOC(c, s.col, sizeof(int32_t) * nnz);
        TRY_ALLOC(c, s.order, sizeof(int32_t) * s.nrows);
        TRY_ALLOC(c, s.seg_first, sizeof(int32_t) * s.nrows);
        if (has_y) TRY_ALLOC(c, s.y, sizeof(float) * nnz);
        if (has_a) TRY_ALLOC(c, s.a, sizeof(float) * nnz);
    }
    TRY_ALLOC(c, is.slot, sizeof(int32_t) * nnz);
    TRY_ALLOC(c, c->yhat, sizeof(float) * nnz);
    TRY_ALLOC(c, c->pred, sizeof(float) * nnz);

    // observations on the device (temporary copies when they come from the host)
    const int32_t *du = S->user, *di = S->item;
    const float *dy = S->y, *da = S->alpha;
    // (counted against the budget while held; freed once the index is built)
    std::vector<std::pair<void*, size_t>> tmp;
    struct TmpFree {
        ials_ctx* c;
        std::vector<std::pair<void*, size_t>>& v;
        ~TmpFree() {
            (void)hipStreamSynchronize(c->stream);
            for (auto& pb : v) ials::tmp_free(c, pb.first, pb.second);
        }
    } tmp_free{c, tmp};
    if (S->memkind == IALS_MEM_HOST && nnz > 0) {
        auto up = [&](const void* src, size_t bytes, void** dst) -> ials_status {
            hipError_t e = ials::tmp_alloc(c, dst, bytes);
            if (e != hipSuccess) {
                g_create_error = "temporary device copy of the observations (" + std::to_string(bytes) +
                                 " bytes) failed: " + hipGetErrorString(e);
                return ials::alloc_status(e);
            }
            tmp.emplace_back(*dst, bytes);
            e = hipMemcpyAsync(*dst, src, bytes, hipMemcpyHostToDevice, c->stream);
            if (e != hipSuccess) {
                g_create_error = std::string("copy of the observations failed: ") + hipGetErrorString(e);
                return IALS_E_HIP;
            }
            return IALS_OK;
        };
        void* p;
        ials_status su = up(S->user, sizeof(int32_t) * nnz, &p);
        if (su != IALS_OK) return su;
        du = (const int32_t*)p;
        su = up(S->item, sizeof(int32_t) * nnz, &p);
        if (su != IALS_OK) return su;
        di = (const int32_t*)p;
        if (has_y) {
            su = up(S->y, sizeof(float) * nnz, &p);
            if (su != IALS_OK) return su;
            dy = (const float*)p;
        }
        if (has_a) {
            su = up(S->alpha, sizeof(float) * nnz, &p);
            if (su != IALS_OK) return su;
            da = (const float*)p;
        }
    }
    {
        ials_status st = ials::build_index(c, du, di, dy, da);
        if (st != IALS_OK) {
            g_create_error = c->err;
            return st;
        }
    }

    // work buffers of the passes
    const int64_t nmax = std::max<int64_t>(c->U, c->I);
    TRY_ALLOC(c, c->G, sizeof(float) * c->d * c->B);
    TRY_ALLOC(c, c->Dmat, sizeof(float) * c->B * c->B);
    TRY_ALLOC(c, c->dtiles, sizeof(float) * 256 * (c->B / 16) * (c->B / 16 + 1) / 2);
    TRY_ALLOC(c, c->R0, sizeof(float) * nmax * c->B);
    TRY_ALLOC(c, c->fb_list, sizeof(int32_t) * nmax);
    size_t gp = 0;
    for (int32_t n : {c->U, c->I})
        for (int32_t nc : {c->B, c->d}) gp = std::max(gp, ials::gram_part_floats_needed(n, c->d, nc, c->precision == IALS_PREC_BF16));
    c->gram_part_floats = gp;
    TRY_ALLOC(c, c->gram_part, sizeof(float) * gp);
    const int64_t nseg = std::max(us.nseg, is.nseg);
    if (nseg > 0) TRY_ALLOC(c, c->seg_part, sizeof(float) * nseg * ials::seg_part_floats_per_segment(c->B));
    if (c->B > 64) TRY_ALLOC(c, c->fb_scratch, sizeof(double) * ials::big_fallback_doubles(c->B));
    // loss scratch: one double per user, then float64 Gramian partials (<= 256 MB)
    const size_t dd = (size_t)c->d * c->d;
    const size_t chunks = std::max<size_t>(1, std::min<size_t>(64, ((size_t)32 << 20) / dd));
    c->loss_part_len = (size_t)std::max<int64_t>(c->U, 1) + chunks * dd;
    TRY_ALLOC(c, c->loss_part, sizeof(double) * c->loss_part_len);
    TRY_ALLOC(c, c->gram64, sizeof(double) * 2 * dd);
    TRY_ALLOC(c, c->loss_out, sizeof(double) * 4);
    // fold-in: G = H^T H, counters, request scratch and pinned request descriptors
    c->fold = ials::fold_shape(c->I, c->d, c->b);
    TRY_ALLOC(c, c->fold_G, sizeof(float) * dd);
    TRY_ALLOC(c, c->fold_cnt, sizeof(int32_t) * ials::FOLD_CNT_NUM);
    c->fold_ws_cap = ((size_t)1 << 22) + (c->fold.gfac ? 64 * ials::fold_ws_floats(c->fold, 0) : 0);
    TRY_ALLOC(c, c->fold_ws, sizeof(float) * c->fold_ws_cap);
    c->fold_req_cap = 16384;
    {
        void* hp = nullptr;
        TRY_HIP_CREATE(hipHostMalloc(&hp, sizeof(ials::FoldReq) * c->fold_req_cap, hipHostMallocMapped));
        c->owned_host.push_back(hp);
        c->fold_req = static_cast<ials::FoldReq*>(hp);
    }

    c->cur_block = 0;
    if (solver_of(c) == IALS_SOLVER_IALS)
        ials::launch_fill(c->stream, c->yhat, c->nnz, 0.f);
    else
        ials::launch_predict(c, 0, false, c->yhat);
    TRY_HIP_CREATE(hipGetLastError());
    TRY_HIP_CREATE(hipStreamSynchronize(c->stream));
    guard.armed = false;
    *out = c;
    return IALS_OK;
}

}  // namespace

extern "C" {

ials_status ials_create(const ials_config* cfg, const ials_coo* S, float* W, float* H, void* hip_stream,
                        ials_ctx** out) {
    try {
        g_create_error.clear();
        return create_impl(cfg, S, W, H, hip_stream, out);
    } catch (...) {
        g_create_error = "unexpected host exception in ials_create";
        return IALS_E_NOMEM;
    }
}

ials_status ials_destroy(ials_ctx* ctx) {
    if (!ctx) return IALS_E_INVALID;
    free_ctx(ctx);
    return IALS_OK;
}

ials_status ials_set_stream(ials_ctx* c, void* hip_stream) {
    if (check_ctx(c) != IALS_OK) return IALS_E_INVALID;
    hipStream_t ns = (hipStream_t)hip_stream;
    if ((c->flags & IALS_FLAG_GRAPH) && ns == nullptr)
        return fail(c, IALS_E_INVALID, "a context with IALS_FLAG_GRAPH needs a non-NULL stream (graphs are not "
                                       "captured on the NULL stream)");
    if (ns == c->stream) return IALS_OK;
    // work already queued on the old stream finishes before anything is queued on the new
    // one (both touch W, H and the prediction cache); a stream the library made is released
    IALS_HIP_TRY(c, hipStreamSynchronize(c->stream));
    if (c->own_stream) {
        IALS_HIP_TRY(c, hipStreamDestroy(c->stream));
        c->own_stream = false;
    }
    c->stream = ns;
    return IALS_OK;
}

ials_status ials_gramian(ials_ctx* c, int32_t which, int32_t block, float* out) {
    if (check_ctx(c) != IALS_OK) return IALS_E_INVALID;
    if (!out || (which != IALS_MAT_W && which != IALS_MAT_H)) return fail(c, IALS_E_INVALID, "bad gramian arguments");
    const int32_t nblocks = (c->d + c->b - 1) / c->b;
    if (block < -1 || block >= nblocks) return fail(c, IALS_E_INVALID, "block index out of range");
    const float* X = which == IALS_MAT_W ? c->W : c->H;
    const int32_t n = which == IALS_MAT_W ? c->U : c->I;
    try {
        if (block == -1)
            ials::launch_gramian_slab(c, X, n, 0, c->d, c->d, out, false);
        else {
            const int32_t bw = block_width(c, block);
            ials::launch_gramian_slab(c, X, n, block * c->b, bw, bw, out, false);
        }
    } catch (...) {
        return fail(c, IALS_E_HIP, "launch failed");
    }
    IALS_HIP_TRY(c, hipGetLastError());
    return IALS_OK;
}

ials_status ials_block_sweep(ials_ctx* c, int32_t side, int32_t block) {
    if (check_ctx(c) != IALS_OK) return IALS_E_INVALID;
    const int32_t nblocks = (c->d + c->b - 1) / c->b;
    if ((side != IALS_SIDE_USER && side != IALS_SIDE_ITEM) || block < 0 || block >= nblocks)
        return fail(c, IALS_E_INVALID, "bad side or block index");
    return run_pass(c, side, block);
}

ials_status ials_refresh_predictions(ials_ctx* c) {
    if (check_ctx(c) != IALS_OK) return IALS_E_INVALID;
    ials::ProfScope ps(c, IALS_K_PREDICT);
    ials::launch_predict(c, c->cur_block, false, c->yhat);
    IALS_HIP_TRY(c, hipGetLastError());
    return IALS_OK;
}

// The launches of one epoch of Alg. 3.
ials_status launch_epoch(ials_ctx* c) {
    const int32_t nblocks = (c->d + c->b - 1) / c->b;
    {
        ials::ProfScope ps(c, IALS_K_PREDICT);
        if (solver_of(c) == IALS_SOLVER_IALS)
            ials::launch_fill(c->stream, c->yhat, c->nnz, 0.f);  // Alg. 1 needs no predictions
        else
            ials::launch_predict(c, 0, false, c->yhat);
        c->cur_block = 0;
    }
    for (int32_t blk = 0; blk < nblocks; ++blk) {
        ials_status s = run_pass(c, IALS_SIDE_USER, blk);
        if (s != IALS_OK) return s;
        s = run_pass(c, IALS_SIDE_ITEM, blk);
        if (s != IALS_OK) return s;
    }
    return IALS_OK;
}

ials_status ials_epoch(ials_ctx* c, int32_t n_epochs) {
    if (check_ctx(c) != IALS_OK) return IALS_E_INVALID;
    if (n_epochs < 0) return fail(c, IALS_E_INVALID, "n_epochs < 0");
    const bool graph = (c->flags & IALS_FLAG_GRAPH) && !c->prof;
    if (graph && n_epochs > 0 && !c->epoch_exec) {
        const int64_t passes0 = c->passes;
        IALS_HIP_TRY(c, hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal));
        ials_status s = launch_epoch(c);
        hipGraph_t g = nullptr;
        hipError_t e = hipStreamEndCapture(c->stream, &g);
        if (s != IALS_OK) {
            if (g) (void)hipGraphDestroy(g);
            return s;
        }
        if (e != hipSuccess) return fail(c, IALS_E_HIP, std::string("epoch capture failed: ") + hipGetErrorString(e));
        e = hipGraphInstantiate(&c->epoch_exec, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        if (e != hipSuccess) {
            c->epoch_exec = nullptr;
            return fail(c, IALS_E_HIP, std::string("epoch graph instantiation failed: ") + hipGetErrorString(e));
        }
        c->passes = passes0;  // nothing ran during the capture
    }
    const int32_t nblocks = (c->d + c->b - 1) / c->b;
    for (int32_t t = 0; t < n_epochs; ++t) {
        if (graph) {
            IALS_HIP_TRY(c, hipGraphLaunch(c->epoch_exec, c->stream));
            c->cur_block = nblocks - 1;
            c->passes += 2 * nblocks;
        } else {
            ials_status s = launch_epoch(c);
            if (s != IALS_OK) return s;
        }
    }
    IALS_HIP_TRY(c, hipGetLastError());
    return IALS_OK;
}

ials_status ials_loss(ials_ctx* c, double* out_host, double* parts_host) {
    if (check_ctx(c) != IALS_OK) return IALS_E_INVALID;
    if (!out_host) return fail(c, IALS_E_INVALID, "null output");
    ials_status s;
    {
        ials::ProfScope ps(c, IALS_K_LOSS);
        s = ials::launch_loss(c);
    }
    if (s != IALS_OK) return s;
    double parts[4] = {0, 0, 0, 0};
    IALS_HIP_TRY(c, hipMemcpyAsync(parts, c->loss_out, sizeof(double) * 3, hipMemcpyDeviceToHost, c->stream));
    long long cnt[ials::CNT_NUM];
    IALS_HIP_TRY(c, hipMemcpyAsync(cnt, c->counters, sizeof(cnt), hipMemcpyDeviceToHost, c->stream));
    IALS_HIP_TRY(c, hipStreamSynchronize(c->stream));
    const double L = parts[0] + (double)c->alpha0 * parts[1] + (double)c->lambda * parts[2];
    *out_host = L;
    if (parts_host) {
        parts_host[0] = parts[0];
        parts_host[1] = (double)c->alpha0 * parts[1];
        parts_host[2] = (double)c->lambda * parts[2];
    }
    if (cnt[ials::CNT_NOT_SPD] > 0)
        return fail(c, IALS_E_NOT_SPD,
                    std::to_string(cnt[ials::CNT_NOT_SPD]) + " rows had a Hessian that was not SPD in float64");
    if (!std::isfinite(L)) return fail(c, IALS_E_INVALID, "loss is not finite");
    return IALS_OK;
}

ials_status ials_get_csr(ials_ctx* c, int32_t side, int64_t* row_ptr, int32_t* col, int32_t* perm) {
    if (check_ctx(c) != IALS_OK) return IALS_E_INVALID;
    if (side != IALS_SIDE_USER && side != IALS_SIDE_ITEM) return fail(c, IALS_E_INVALID, "bad side");
    const ials::SideIndex& s = c->side[side];
    if (row_ptr)
        IALS_HIP_TRY(c, hipMemcpyAsync(row_ptr, s.ptr, sizeof(int64_t) * (s.nrows + 1), hipMemcpyDeviceToHost, c->stream));
    if (col && c->nnz > 0)
        IALS_HIP_TRY(c, hipMemcpyAsync(col, s.col, sizeof(int32_t) * c->nnz, hipMemcpyDeviceToHost, c->stream));
    if (perm && side == IALS_SIDE_ITEM && c->nnz > 0)
        IALS_HIP_TRY(c, hipMemcpyAsync(perm, s.slot, sizeof(int32_t) * c->nnz, hipMemcpyDeviceToHost, c->stream));
    IALS_HIP_TRY(c, hipStreamSynchronize(c->stream));
    return IALS_OK;
}

ials_status ials_get_predictions(ials_ctx* c, float* out_host) {
    if (check_ctx(c) != IALS_OK) return IALS_E_INVALID;
    if (!out_host) return fail(c, IALS_E_INVALID, "null output");
    if (c->nnz > 0) {
        ials::launch_predict(c, c->cur_block, true, c->pred);
        IALS_HIP_TRY(c, hipGetLastError());
        IALS_HIP_TRY(c, hipMemcpyAsync(out_host, c->pred, sizeof(float) * c->nnz, hipMemcpyDeviceToHost, c->stream));
    }
    IALS_HIP_TRY(c, hipStreamSynchronize(c->stream));
    return IALS_OK;
}

ials_status ials_get_stats(ials_ctx* c, ials_stats* o) {
    if (check_ctx(c) != IALS_OK) return IALS_E_INVALID;
    if (!o) return fail(c, IALS_E_INVALID, "null output");
    long long cnt[ials::CNT_NUM];
    IALS_HIP_TRY(c, hipMemcpyAsync(cnt, c->counters, sizeof(cnt), hipMemcpyDeviceToHost, c->stream));
    IALS_HIP_TRY(c, hipStreamSynchronize(c->stream));
    std::memset(o, 0, sizeof(*o));
    o->nnz = c->nnz;
    o->num_users = c->U;
    o->num_items = c->I;
    o->dim = c->d;
    o->block = c->b;
    o->padded_block = c->B;
    o->long_rows_user = c->side[0].nlong;
    o->long_rows_item = c->side[1].nlong;
    o->segments_user = c->side[0].nseg;
    o->segments_item = c->side[1].nseg;
    o->fallback_rows = cnt[ials::CNT_FALLBACK_ROWS];
    o->passes = c->passes;
    o->device_bytes = c->device_bytes;
    o->peak_device_bytes = c->peak_bytes;
    o->solver = solver_of(c);
    o->foldin_requests = c->fold_requests;
    o->foldin_float64 = c->fold_float64;
    return IALS_OK;
}

ials_status ials_profile_enable(ials_ctx* c, int32_t enable) {
    if (check_ctx(c) != IALS_OK) return IALS_E_INVALID;
    IALS_HIP_TRY(c, hipStreamSynchronize(c->stream));
    if (enable && c->prof_pool.empty()) {
        constexpr size_t kPairs = 16384;
        c->prof_pool.resize(2 * kPairs, nullptr);
        c->prof_kind.resize(kPairs, 0);
        for (auto& e : c->prof_pool) IALS_HIP_TRY(c, hipEventCreate(&e));
    }
    c->prof = enable != 0;
    c->prof_used = 0;
    for (int k = 0; k < IALS_K_NUM; ++k) {
        c->prof_ms[k] = 0.0;
        c->prof_count[k] = 0;
    }
    return IALS_OK;
}

ials_status ials_profile_read(ials_ctx* c, double* total_ms, int64_t* launches) {
    if (check_ctx(c) != IALS_OK) return IALS_E_INVALID;
    IALS_HIP_TRY(c, hipStreamSynchronize(c->stream));
    for (size_t i = 0; i < c->prof_used; ++i) {
        float ms = 0.f;
        IALS_HIP_TRY(c, hipEventElapsedTime(&ms, c->prof_pool[2 * i], c->prof_pool[2 * i + 1]));
        c->prof_ms[c->prof_kind[i]] += ms;
        c->prof_count[c->prof_kind[i]] += 1;
    }
    c->prof_used = 0;
    for (int k = 0; k < IALS_K_NUM; ++k) {
        if (total_ms) total_ms[k] = c->prof_ms[k];
        if (launches) launches[k] = c->prof_count[k];
        c->prof_ms[k] = 0.0;
        c->prof_count[k] = 0;
    }
    return IALS_OK;
}

ials_status ials_foldin(ials_ctx* c, int32_t n_req, const int64_t* req_ptr, const int32_t* items, const float* y,
                        int32_t passes, float* W_out) {
    if (check_ctx(c) != IALS_OK) return IALS_E_INVALID;
    if (n_req < 0 || passes < 0 || passes > 1000) return fail(c, IALS_E_INVALID, "need n_req >= 0 and 0 <= passes <= 1000");
    if (n_req == 0) return IALS_OK;
    if (!req_ptr || !W_out) return fail(c, IALS_E_INVALID, "null req_ptr or W_out");
    if (req_ptr[0] != 0) return fail(c, IALS_E_INVALID, "req_ptr[0] must be 0");
    for (int32_t r = 0; r < n_req; ++r)
        if (req_ptr[r + 1] < req_ptr[r] || req_ptr[r + 1] - req_ptr[r] > (int64_t)INT32_MAX)
            return fail(c, IALS_E_INVALID, "req_ptr must be non-decreasing with requests below 2^31 items");
    if (req_ptr[n_req] > 0 && !items) return fail(c, IALS_E_INVALID, "null items");
    if (c->b > 64) return fail(c, IALS_E_INVALID, "fold-in needs block <= 64");
    if (c->fold_G_passes != c->passes) {
        ials::launch_gramian_slab(c, c->H, c->I, 0, c->d, c->d, c->fold_G, false);
        c->fold_G_passes = c->passes;
    }
    IALS_HIP_TRY(c, hipMemsetAsync(c->fold_cnt, 0, sizeof(int32_t) * ials::FOLD_CNT_NUM, c->stream));
    int32_t r = 0;
    while (r < n_req) {
        int32_t m = 0;
        size_t used = 0;
        while (r + m < n_req && m < c->fold_req_cap) {
            const int64_t lo = req_ptr[r + m], n = req_ptr[r + m + 1] - lo;
            const size_t need = ials::fold_ws_floats(c->fold, n);
            if (used + need > c->fold_ws_cap) break;
            ials::FoldReq& q = c->fold_req[m];
            q.items = items + lo;
            q.y = y ? y + lo : nullptr;
            q.ws = c->fold_ws + used;
            q.out = W_out + (size_t)(r + m) * c->d;
            q.st = nullptr;
            q.n = (int32_t)n;
            q.copy = 0;
            used += need;
            ++m;
        }
        if (m == 0)
            return fail(c, IALS_E_INVALID, "request " + std::to_string(r) + " has more items than the fold-in scratch holds");
        void* dreq = nullptr;
        IALS_HIP_TRY(c, hipHostGetDevicePointer(&dreq, c->fold_req, 0));
        IALS_HIP_TRY(c, ials::launch_foldin(c->stream, c->fold, c->H, c->fold_G, c->alpha0, c->lambda, c->tau, passes,
                                            static_cast<const ials::FoldReq*>(dreq), m, c->fold_cnt));
        // the descriptors and the scratch are reused by the next chunk
        IALS_HIP_TRY(c, hipStreamSynchronize(c->stream));
        r += m;
    }
    int32_t cnt[ials::FOLD_CNT_NUM];
    IALS_HIP_TRY(c, hipMemcpyAsync(cnt, c->fold_cnt, sizeof(cnt), hipMemcpyDeviceToHost, c->stream));
    IALS_HIP_TRY(c, hipStreamSynchronize(c->stream));
    c->fold_requests += n_req;
    c->fold_float64 += cnt[ials::FOLD_CNT_FLOAT64];
    if (cnt[ials::FOLD_CNT_BAD_ID] > 0)
        return fail(c, IALS_E_INVALID, std::to_string(cnt[ials::FOLD_CNT_BAD_ID]) + " requests hold item ids out of range");
    if (cnt[ials::FOLD_CNT_NOT_SPD] > 0)
        return fail(c, IALS_E_NOT_SPD, std::to_string(cnt[ials::FOLD_CNT_NOT_SPD]) +
                                           " requests had a block Hessian that was not SPD in float64");
    return IALS_OK;
}

const char* ials_last_error(const ials_ctx* c) {
    if (!c) return g_create_error.c_str();
    return c->err.c_str();
}

const char* ials_version(void) { return "libials 0.1 (gfx950)"; }

}  // extern "C"
