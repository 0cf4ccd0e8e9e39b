/*
 * libials -- iALS++ block-coordinate sweep on AMD Instinct MI355X (gfx950).
 *
 * Method: Rendle, Krichene, Zhang, Koren, "iALS++: Speeding up Matrix
 * Factorization with Subspace Optimization" (arXiv 2110.14044).  Notation:
 *   S      observations (u, i, y, alpha) (sec. 2), y = alpha = 1 unless given;
 *   W, H   user (U x d) and item (I x d) embeddings, yhat(u,i) = <w_u, h_i> (eq. 1);
 *   L      sum_S alpha (yhat - y)^2 + alpha0 sum_{u,i} yhat^2 + lambda (|W|^2 + |H|^2) (eq. 2);
 *   pi     a block of b consecutive coordinates; the partition is the ascending
 *          blocks [0,b), [b,2b), ... (the last one shorter when b does not divide d);
 *   G      Gramian of the fixed side (eq. 4) and its partial form d x |pi| (eq. 7).
 *
 * Conventions shared by every call:
 *   - every call returns ials_status: 0 (IALS_OK) or a negative error code; no
 *     C++ exception crosses this boundary; ials_last_error() describes the last error;
 *   - matrices are row-major float32 in device memory unless stated otherwise;
 *   - W and H are BORROWED: the caller allocates them on the device (U*d and I*d
 *     floats), keeps them alive until ials_destroy, and the library updates them
 *     in place;
 *   - every other buffer the library needs is allocated by ials_create and
 *     released by ials_destroy; no call in between allocates device memory;
 *   - work is enqueued asynchronously on the stream given to ials_create; only
 *     ials_create, ials_loss, ials_foldin, the ials_get_* calls and ials_destroy
 *     synchronise with it.  A device fault surfaces at the next synchronising
 *     call as IALS_E_HIP;
 *   - one context must not be used from two host threads at the same time.
 */
#ifndef IALS_H_
#define IALS_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#if defined(__GNUC__)
#define IALS_API __attribute__((visibility("default")))
#else
#define IALS_API
#endif

typedef enum {
    IALS_OK = 0,
    IALS_E_INVALID = -1, /* bad argument: sizes, ids out of range, repeated (u,i), null pointer */
    IALS_E_NOMEM = -2,   /* device allocation failed or exceeds the configured budget */
    IALS_E_HIP = -3,     /* a HIP runtime call failed (including an earlier asynchronous fault) */
    IALS_E_NOT_SPD = -4, /* a block Hessian was not positive definite even in float64 */
    IALS_E_BUSY = -5,    /* serving: request not admitted now (no free slot or memory); retry */
    IALS_E_STATE = -6    /* call not valid in the object's current state */
} ials_status;

typedef enum { IALS_SIDE_USER = 0, IALS_SIDE_ITEM = 1 } ials_side;
typedef enum { IALS_MAT_W = 0, IALS_MAT_H = 1 } ials_matrix;
typedef enum { IALS_MEM_HOST = 0, IALS_MEM_DEVICE = 1 } ials_memkind;

/* Arithmetic of the contractions (Gramian, dense term, gathered block Hessians).
 * FP32: float32 operands on the matrix cores, float32 accumulation.
 * BF16: bfloat16 operands (round-to-nearest-even from float32) on the matrix
 *       cores with float32 accumulation; gradients, solves and updates stay float32. */
typedef enum { IALS_PREC_FP32 = 0, IALS_PREC_BF16 = 1 } ials_precision;

/* IALS_FLAG_GRAPH: ials_epoch captures the launches of one epoch into a HIP graph
 * on its first call and replays the graph afterwards (an epoch always runs the
 * same launch sequence).  The context's stream must not be the NULL stream; if it
 * is, ials_create makes a private stream for the context.  While profiling is on
 * (ials_profile_enable) epochs run launch by launch. */
enum { IALS_FLAG_GRAPH = 1u };
/* Row dealing of the block-pass kernels (tuning; results do not depend on it):
 * IALS_FLAG_DEAL_QUEUE: wavefronts take rows from a shared atomic queue;
 * IALS_FLAG_DEAL_STATIC: rows are dealt round-robin in decreasing length order.
 * Neither: static. */
enum { IALS_FLAG_DEAL_QUEUE = 2u, IALS_FLAG_DEAL_STATIC = 4u };

/* The passes a block size runs (sec. 3 and 4: iALS and iCD are the b = d and b = 1 ends of
 * iALS++).  IALS_SOLVER_BLOCK: the block Newton steps of Alg. 3.  IALS_SOLVER_IALS (b = d):
 * Alg. 1, every row solved against its dense normal equations (eq. 3) with no prediction
 * cache and no dense gradient term; the rows of the side being solved are overwritten (zeroed
 * first) during the pass.  IALS_SOLVER_ICD (b = 1): Alg. 2, scalar coordinate descent with
 * the column g of the Gramian (no padded block, no factorisation). */
typedef enum { IALS_SOLVER_BLOCK = 0, IALS_SOLVER_IALS = 1, IALS_SOLVER_ICD = 2 } ials_solver;

typedef struct {
    int32_t num_users;          /* U >= 1 */
    int32_t num_items;          /* I >= 1 */
    int32_t dim;                /* d >= 1 */
    int32_t block;              /* b, 1 <= b <= min(d, 256): b = 1 runs coordinate descent
                                   (Alg. 2), b = d full-row solves (Alg. 1); blocks of 65..128
                                   are padded to 128 (one wavefront per row), of 129..256 to
                                   256 (one workgroup per row) */
    float alpha0;               /* weight of the all-pairs term, >= 0 */
    float lambda;               /* L2 weight, > 0 */
    int32_t precision;          /* ials_precision */
    float chol_fallback_ratio;  /* tau: a row whose smallest float32 pivot (the diagonal of D
                                   in Hess = L D L^T, i.e. the squared Cholesky diagonal) is
                                   below tau times the largest diagonal entry of its block
                                   Hessian (their ratio bounds 1 / condition number from
                                   above), or whose pivots are not all positive, is
                                   refactored in float64; <= 0 selects 1e-4; >= 1 redoes
                                   every row */
    uint32_t flags;             /* IALS_FLAG_* bits */
    uint32_t seg_len;           /* rows longer than this are accumulated in segments of this many
                                   observations (split-K); a multiple of 64 in [256, 65536];
                                   0 selects 512 */
    uint64_t hbm_budget;        /* upper bound on the library's device bytes held at any time,
                                   the temporaries of ials_create included; 0 = no bound */
    uint32_t gram_split;        /* split-K of the per-pass Gramian slab (eq. 7): the number of
                                   workgroups its row chunks and output tiles are sized for, a
                                   power of two in [64, 2048]; 0 selects 512.  The chunk partials
                                   are added in float64 in chunk order, so a different split
                                   rounds differently (results stay deterministic per split) */
    uint32_t reserved;          /* 0 */
} ials_config;

typedef struct {
    int64_t nnz;          /* |S| >= 0 */
    const int32_t* user;  /* [nnz] user id of each observation, 0 <= u < U */
    const int32_t* item;  /* [nnz] item id, 0 <= i < I; each (u, i) at most once */
    const float* y;       /* [nnz] labels, or NULL for all ones */
    const float* alpha;   /* [nnz] weights > 0, or NULL for all ones */
    int32_t memkind;      /* ials_memkind of the four arrays above */
    int32_t reserved;
} ials_coo;

typedef struct ials_ctx ials_ctx;

typedef struct {
    int64_t nnz;
    int32_t num_users, num_items, dim, block, padded_block;
    int32_t long_rows_user, long_rows_item;  /* rows split into segments */
    int64_t segments_user, segments_item;
    int64_t fallback_rows;     /* rows refactored in float64 since create */
    int64_t passes;            /* block passes run since create */
    uint64_t device_bytes;     /* library-owned device memory */
    int64_t foldin_requests;   /* rows folded in by ials_foldin since create */
    int64_t foldin_float64;    /* of those, rows redone in float64 */
    uint64_t peak_device_bytes; /* most device memory held at once by the library, including the
                                   temporaries of ials_create; an hbm_budget below it makes
                                   ials_create fail with IALS_E_NOMEM */
    int32_t solver;            /* ials_solver the block size selected */
    int32_t reserved;
} ials_stats;

/*
 * Create a training context (sec. 2 problem; Alg. 3 state).  Validates the
 * configuration and the observations, copies S into library-owned device
 * memory, builds the user-major and item-major observation indices and
 * computes yhat from the current W and H.  hip_stream is a hipStream_t (NULL =
 * the default stream).  On success *out owns every allocation; on failure
 * nothing is leaked and *out is NULL.  Synchronising.
 */
IALS_API ials_status ials_create(const ials_config* cfg, const ials_coo* S, float* W, float* H,
                        void* hip_stream, ials_ctx** out);

/* Release everything ials_create allocated.  Never frees W or H.  Synchronising. */
IALS_API ials_status ials_destroy(ials_ctx* ctx);

/*
 * Partial Gramian (eq. 7) of the current W or H: out = X^T X[:, pi] (d x |pi|,
 * row-major) for block index `block` (pi = [block*b, min(block*b+b, d))), or the
 * full Gramian X^T X (d x d, eq. 4) for block = -1.  out is device memory of at
 * least d*|pi| (or d*d) floats.  Per-chunk float32 partial sums are combined in
 * float64.  Asynchronous.
 */
IALS_API ials_status ials_gramian(ials_ctx* ctx, int32_t which, int32_t block, float* out);

/*
 * One pass of Alg. 3 for one block and one side: side USER updates w_{u,pi}
 * for every user against the current H; side ITEM updates h_{i,pi} against the
 * current W.  Each row gets one Newton step on its block (sec. 4, eq. 8-9:
 * gradient from the cached yhat and the partial Gramian, Hessian from the
 * gathered partner sub-vectors), an LDL^T solve, the update and the yhat
 * patch.  yhat must be current (create, ials_epoch and this call keep it so).
 * Asynchronous.
 */
IALS_API ials_status ials_block_sweep(ials_ctx* ctx, int32_t side, int32_t block);

/*
 * n_epochs iterations of Alg. 3: recompute yhat (eq. 1), then for every block in
 * ascending order the user pass followed by the item pass.  Asynchronous.
 */
IALS_API ials_status ials_epoch(ials_ctx* ctx, int32_t n_epochs);

/*
 * Recompute yhat = <w_u, h_i> for every observation from the current W and H
 * (the first step of an epoch in Alg. 3).  Asynchronous.
 */
IALS_API ials_status ials_refresh_predictions(ials_ctx* ctx);

/*
 * Loss of eq. 2 for the current W and H, with predictions recomputed from W
 * and H (not the cache) and accumulated in float64; the all-pairs term uses
 * <W^T W, H^T H>_F with both Gramians formed in float64.  parts (nullable, host,
 * 3 doubles) receives the observed term, the alpha0 term and the lambda term.
 * Synchronising; returns IALS_E_INVALID if the result is not finite.
 */
IALS_API ials_status ials_loss(ials_ctx* ctx, double* out_host, double* parts_host);

/* Copy the observation index to host buffers (any may be NULL):
 * side USER: row_ptr[U+1], col[nnz] (item ids); perm ignored.
 * side ITEM: row_ptr[I+1], col[nnz] (user ids), perm[nnz] = user-major slot of
 * each item-major slot.  Synchronising. */
IALS_API ials_status ials_get_csr(ials_ctx* ctx, int32_t side, int64_t* row_ptr, int32_t* col, int32_t* perm);

/* Copy the cached predictions (user-major slot order, nnz floats) to the host. Synchronising. */
IALS_API ials_status ials_get_predictions(ials_ctx* ctx, float* out_host);

/* Counters and sizes.  Synchronising. */
IALS_API ials_status ials_get_stats(ials_ctx* ctx, ials_stats* out);

/*
 * Fold-in (sec. 4, Alg. 3 for a single new row with the item side fixed; eq. 3
 * is its limit): for each request r, a new user who observed the items
 * items[req_ptr[r] .. req_ptr[r+1]) (labels y, or all ones; weights 1), start
 * from w = 0 and run `passes` sweeps over the blocks in ascending order, each a
 * block Newton step against the context's current H and G = H^T H (eq. 8-9 with
 * the predictions of this row only).  The result row r is written to
 * W_out[r*d .. r*d+d).
 *   req_ptr  HOST array of n_req+1 non-decreasing offsets, req_ptr[0] = 0;
 *   items    DEVICE int32 [req_ptr[n_req]], ids in [0, I);
 *   y        DEVICE float [req_ptr[n_req]] labels, or NULL for all ones;
 *   W_out    DEVICE float [n_req * d], caller-owned.
 * Every request's block Hessians are factored once (H does not change during a
 * fold-in) in float32; a request whose pivots fail the chol_fallback_ratio test
 * is redone entirely in float64.  Requests are independent: a request's result
 * does not depend on the other requests of the call.  G is re-formed when a
 * training pass has run since the previous fold-in (changes made to H outside
 * the library after that are not seen).  Runs on the context's stream in
 * chunks that fit the fold-in scratch allocated by ials_create; returns
 * IALS_E_INVALID for bad offsets, an item id out of range (detected on the
 * device; the call then leaves W_out undefined) or a request longer than the
 * scratch, IALS_E_NOT_SPD if a request failed even in float64 (its row is NaN).
 * Synchronising.
 */
IALS_API ials_status ials_foldin(ials_ctx* ctx, int32_t n_req, const int64_t* req_ptr, const int32_t* items,
                                 const float* y, int32_t passes, float* W_out);

/* Kernel families timed by the profiling hooks below (index into the arrays). */
typedef enum {
    IALS_K_PREDICT = 0,       /* yhat recompute at the start of an epoch (eq. 1) */
    IALS_K_GRAM_USER = 1,     /* partial Gramian of H for a user pass (eq. 7) */
    IALS_K_GRAM_ITEM = 2,     /* partial Gramian of W for an item pass */
    IALS_K_DENSE_USER = 3,    /* alpha0 w_u G^pi + lambda w_{u,pi} for every user (eq. 8) */
    IALS_K_DENSE_ITEM = 4,
    IALS_K_SEG_USER = 5,      /* partial Hessians/gradients of long-row segments */
    IALS_K_SEG_ITEM = 6,
    IALS_K_ROWS_USER = 7,     /* gather + Hessian + LDL^T solve + update + yhat patch per row */
    IALS_K_ROWS_ITEM = 8,
    IALS_K_FALLBACK_USER = 9, /* float64 redo of rejected factorisations */
    IALS_K_FALLBACK_ITEM = 10,
    IALS_K_PATCH_USER = 11,   /* yhat patch of long-row segments */
    IALS_K_PATCH_ITEM = 12,
    IALS_K_LOSS = 13,
    IALS_K_ROWS_USER_MOVE = 14, /* a row pass that also moves the prediction cache to its block */
    IALS_K_ROWS_ITEM_MOVE = 15,
    IALS_K_NUM = 16
} ials_kernel;

/* Turn per-kernel timing on (1) or off (0).  While on, every launch of the
 * families above is bracketed by HIP events recorded on the context's stream
 * (event objects are created here, not device memory).  Turning it on clears
 * the accumulated times. */
IALS_API ials_status ials_profile_enable(ials_ctx* ctx, int32_t enable);

/* Accumulated time (ms, host array of IALS_K_NUM) and launch count per family
 * since profiling was enabled or last read; resets the accumulators.
 * Synchronising. */
IALS_API ials_status ials_profile_read(ials_ctx* ctx, double* total_ms, int64_t* launches);

/* Enqueue subsequent work of ctx on another stream (hipStream_t; NULL = default).
 * Waits for the work already queued on the current stream first, so that the two
 * streams never run passes over W, H and the prediction cache at the same time.
 * A stream that ials_create made for the context is destroyed here.  IALS_E_INVALID
 * for a NULL stream on a context with IALS_FLAG_GRAPH.  Synchronising. */
IALS_API ials_status ials_set_stream(ials_ctx* ctx, void* hip_stream);

/* Text of the last error on ctx (or of the last failed ials_create when ctx is NULL). */
IALS_API const char* ials_last_error(const ials_ctx* ctx);

/*
 * Fold-in server: continuous batching of fold-in requests (the fold-in above)
 * against a resident item table.  The server keeps G = H^T H on the device,
 * admits each request into a slot and a region of its device arena (the HBM
 * budget), and a worker thread launches everything admitted as one batch on
 * the next free stream while earlier batches are still running, so requests
 * that arrive while others are on the GPU start as soon as a stream is free.
 * Each request runs in its own workgroup with the same arithmetic whatever the
 * batch holds: a result is bitwise the same alone or in any mix.
 */
typedef struct ials_server ials_server;

typedef struct {
    int32_t num_items;          /* I >= 1, rows of H */
    int32_t dim;                /* d >= 1 */
    int32_t block;              /* b, 1 <= b <= min(d, 64) */
    float alpha0;               /* >= 0 */
    float lambda;               /* > 0 */
    int32_t precision;          /* ials_precision (IALS_PREC_FP32) */
    int32_t passes;             /* sweeps per request, 0..1000 */
    int32_t max_slots;          /* requests admitted at once (queued, running or unpolled), >= 1 */
    int32_t streams;            /* batches in flight at once, 1..8; 0 selects 4 */
    float chol_fallback_ratio;  /* tau as in ials_config; <= 0 selects 1e-4 */
    uint64_t hbm_budget;        /* bytes of the device arena for request state; 0 selects 64 MiB */
} ials_server_config;

typedef struct {
    int64_t submitted;          /* admitted requests */
    int64_t rejected_busy;      /* submissions answered IALS_E_BUSY */
    int64_t completed;          /* requests whose batch finished */
    int64_t polled;             /* results handed out by ials_server_poll */
    int64_t batches;            /* batches launched */
    int64_t max_batch;          /* largest batch */
    int64_t float64_requests;   /* polled results that were redone in float64 */
    int64_t not_spd_requests;   /* polled results that failed in float64 */
    int32_t admitted;           /* requests holding a slot now */
    int32_t in_flight;          /* batches on the device now */
    uint64_t arena_bytes;       /* hbm_budget */
    uint64_t bytes_in_use;      /* arena bytes held by admitted requests */
    uint64_t bytes_peak;
} ials_server_stats;

/* Create a server on the current device.  H is a DEVICE float [I x d] table,
 * BORROWED: it must stay alive and unchanged until ials_server_destroy.
 * Allocates the arena (hbm_budget bytes of device memory and as much pinned
 * host memory), G, one stream per batch in flight, and starts the worker
 * thread.  Synchronising.  On failure *out is NULL and
 * ials_server_last_error(NULL) describes the error. */
IALS_API ials_status ials_server_create(const ials_server_config* cfg, const float* H, ials_server** out);

/* Submit one request: n >= 0 HOST item ids (and HOST labels y, or NULL for ones),
 * copied before the call returns; tag is returned with the result.  Returns
 * IALS_OK if admitted, IALS_E_BUSY if every slot is taken or the arena has no
 * room for it now (nothing was queued: retry after polling), IALS_E_INVALID
 * for an id out of range or a request larger than the whole arena, IALS_E_STATE
 * once the worker has failed.  Thread-safe; never blocks on the device. */
IALS_API ials_status ials_server_submit(ials_server* srv, int32_t n, const int32_t* items, const float* y,
                                        uint64_t tag);

/* Hand out up to max finished results: tags[k], the row w_out[k*d .. k*d+d)
 * (HOST) and status[k] (nullable; 0 = float32 path, 1 = redone in float64,
 * 2 = not SPD in float64: row is NaN).  Waits up to wait_us microseconds for a
 * first result when none is ready.  *n_done receives the count.  Frees the
 * results' slots and arena regions.  Thread-safe.  Returns IALS_E_HIP once a
 * device error has stopped the worker (results finished before it are still
 * handed out). */
IALS_API ials_status ials_server_poll(ials_server* srv, int32_t max, int32_t wait_us, uint64_t* tags, float* w_out,
                                      int32_t* status, int32_t* n_done);

/* Counters of the server.  Thread-safe. */
IALS_API ials_status ials_server_stats_get(ials_server* srv, ials_server_stats* out);

/* Stop the worker (requests not yet launched are dropped, running batches are
 * waited for) and release everything the server allocated.  Never frees H. */
IALS_API ials_status ials_server_destroy(ials_server* srv);

/* Text of the last error of srv (or of the last failed ials_server_create when srv is NULL). */
IALS_API const char* ials_server_last_error(const ials_server* srv);

/*
 * Top-k recommendation (sec. 2: items are ranked for a user by yhat(u, i) = <w_u, h_i>, eq. 1;
 * sec. 5.1 ranks, for each evaluated user, all items not given for that user).  For every user
 * u < n_users, out_ids[u*k .. u*k+k) receives the k items of largest score among those not
 * excluded for u, ordered by score descending and equal scores by id ascending, and
 * out_scores the float32 scores (the matrix-core product of W and H); when fewer than k items
 * are eligible the tail holds id -1 and score -inf.  Scores that are NaN are not eligible.
 *   W        DEVICE float [n_users * d] row-major, 16-byte aligned (a batch of user rows);
 *   H        DEVICE float [n_items * d] row-major, 16-byte aligned (may be NULL when n_items
 *            is 0);  d a multiple of 4;
 *   excl_ptr DEVICE int64 [n_users + 1] offsets into excl_idx, or NULL (nothing excluded);
 *   excl_idx DEVICE int32 item ids excluded per user (ids outside [0, n_items) are ignored);
 *   k        1 <= k <= 512;
 *   out_ids  DEVICE int32 [n_users * k];  out_scores DEVICE float [n_users * k] or NULL;
 *   score_buffer_bytes  bound of the score buffer (users are scored in batches whose scores
 *            fit it; 0 selects 1 GiB); the buffer is allocated and freed on the stream;
 *   stream   hipStream_t (NULL: the default stream).
 * Asynchronous (returns after enqueueing); IALS_E_INVALID for bad sizes or pointers,
 * IALS_E_NOMEM if the score buffer cannot be allocated.  Error text: ials_rank_last_error().
 */
IALS_API ials_status ials_rank_topk(const float* W, int64_t n_users, const float* H, int32_t n_items, int32_t d,
                                    const int64_t* excl_ptr, const int32_t* excl_idx, int32_t k, int32_t* out_ids,
                                    float* out_scores, int64_t score_buffer_bytes, void* stream);

/*
 * ials_rank_topk for callers that cannot allocate device memory (code under HIP graph
 * capture, serving loops, hosts that forbid hipMalloc): the same arguments, kernels and
 * results, with the score buffer taken from a fixed array of 64 MiB in device memory that
 * the library holds on every GPU it runs on until the process ends (users are scored in
 * batches whose scores fit it).  Allocates nothing and frees nothing.  Calls that overlap on
 * one GPU (several streams or host threads at once) share that array and race; issue them
 * one after another.  IALS_E_INVALID, before any device work, for the arguments
 * ials_rank_topk rejects and for n_items above 16,777,216 (one user's scores would not fit);
 * IALS_E_HIP if the array's device address cannot be obtained.  stream must belong to the
 * current device.  Asynchronous.
 */
IALS_API ials_status ials_rank_topk_noalloc(const float* W, int64_t n_users, const float* H, int32_t n_items,
                                            int32_t d, const int64_t* excl_ptr, const int32_t* excl_idx, int32_t k,
                                            int32_t* out_ids, float* out_scores, void* stream);

/*
 * Ranking metrics of the holdout evaluation (sec. 5.1 names Recall@k and NDCG@k; the
 * definitions are those of the protocol it follows).  For ranked lists ids [n_users * k] (id -1:
 * no item) and held-out items T_u = hold_idx[hold_ptr[u] .. hold_ptr[u+1]) (DEVICE, ids
 * ascending within a user), metric m (kind 0: Recall, kind 1: NDCG, at k_m = ks[m] <= k) is
 *   Recall@k_m = hits in the first k_m / min(k_m, |T_u|)
 *   NDCG@k_m   = sum over hit ranks r <= k_m of 1/log2(r+1), over sum_{r <= min(k_m, |T_u|)} 1/log2(r+1)
 * in float64, written to per_user [n_users * n_metrics] (DEVICE, caller-owned; NaN for a
 * user with no held-out item).  sums_host[m] and counts_host[m] (HOST) receive the sum over
 * users with a value and their number.  kinds and ks are HOST arrays of n_metrics <= 64.
 * Held-out lists that are not ascending give undefined values (no invalid memory access).
 * Synchronising.
 */
IALS_API ials_status ials_rank_metrics(const int32_t* ids, int64_t n_users, int32_t k, const int64_t* hold_ptr,
                                       const int32_t* hold_idx, int32_t n_metrics, const int32_t* kinds,
                                       const int32_t* ks, double* per_user, double* sums_host, int64_t* counts_host,
                                       void* stream);

/* Text of the last error of ials_rank_topk / ials_rank_metrics on this thread. */
IALS_API const char* ials_rank_last_error(void);

/* Library version string. */
IALS_API const char* ials_version(void);

#ifdef __cplusplus
}
#endif

#endif /* IALS_H_ */
