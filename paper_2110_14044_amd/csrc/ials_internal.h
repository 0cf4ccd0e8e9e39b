// Internal declarations of libials (gfx950).  Not part of the public boundary.
#pragma once

#include <hip/hip_runtime.h>

#include <atomic>
#include <cstdint>
#include <string>
#include <vector>

#include "ials.h"

namespace ials {

typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef short shortx4 __attribute__((ext_vector_type(4)));

constexpr int kWave = 64;

// Sum over the 16 lanes of each row of a wavefront (lanes 16r .. 16r + 15), returned in all 16:
// DPP rotations within the row by 8, 4, 2 and 1 lanes.  Each step adds a value that equals the
// xor-partner's (the partial sums are periodic in the row), so every lane ends with the same
// value as an xor butterfly, without a trip through LDS.
__device__ inline float row_sum16(float s) {
    s += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(s), 0x128, 0xf, 0xf, false));  // row_ror:8
    s += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(s), 0x124, 0xf, 0xf, false));  // row_ror:4
    s += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(s), 0x122, 0xf, 0xf, false));  // row_ror:2
    s += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(s), 0x121, 0xf, 0xf, false));  // row_ror:1
    return s;
}
// Rows longer than the context's segment length (512 by default) are split into
// segments of that many observations, each accumulated by its own wavefront (or
// workgroup), then reduced in a fixed order.
constexpr int kSegLenDefault = 512;
constexpr int kGramSplitDefault = 512;

// Device-side counters/flags block (int64), zeroed at create.
enum Counter : int {
    CNT_FALLBACK_ROWS = 0,  // rows refactored in float64
    CNT_NOT_SPD = 1,        // rows not SPD even in float64
    CNT_BAD_INPUT = 2,      // create-time validation failures
    CNT_DUPLICATE = 3,      // repeated (u, i) pairs
    CNT_NUM = 8
};

// Work-queue cursors (int32), reset by the Gramian reduction kernel of each pass.
enum Cursor : int { CUR_ROWS = 0, CUR_SEGS = 1, CUR_PATCH = 2, CUR_FALLBACK = 3, CUR_FB_LIST = 4, CUR_NUM = 8 };

struct SideIndex {
    int32_t nrows = 0;
    int64_t* ptr = nullptr;       // [nrows+1]
    int32_t* col = nullptr;       // [nnz] partner ids
    int32_t* slot = nullptr;      // [nnz] yhat position (item side only; null = identity)
    float* y = nullptr;           // [nnz] labels in this side's order (null = ones)
    float* a = nullptr;           // [nnz] weights in this side's order (null = ones)
    int32_t* order = nullptr;     // [nrows] rows by decreasing length
    int32_t* seg_first = nullptr; // [nrows] first segment of a long row, -1 otherwise
    int32_t* seg_row = nullptr;   // [nseg]
    int64_t* seg_lo = nullptr;    // [nseg]
    int64_t* seg_hi = nullptr;    // [nseg]
    int32_t* seg_order = nullptr; // [nseg] segments by their first partner id (processing order)
    int32_t nseg = 0;
    int32_t nlong = 0;
    int64_t max_len = 0;
};

// Arguments of the block-pass kernels (one pass: one side, one block pi = [p0, p0+bw)).
struct SweepArgs {
    const int64_t* ptr;
    const int32_t* col;
    const int32_t* slot;  // cache position per observation (null: identity)
    const float* y;       // labels in this side's order (null: ones)
    const float* a;       // weights in this side's order (null: ones)
    float* X;             // side being updated, N x d
    const float* Xo;      // fixed side
    float* cache;         // prediction cache (user-major positions)
    const float* R0;      // N x B
    const float* Dmat;    // B x B
    float* dtiles;        // the Hessian start in accumulator layout (NTL x 64 x 4)
    int32_t d, p0, bw, nrows;
    int32_t pc, bwc;      // the block the cache is relative to when the pass starts
    int32_t cur_full;     // that block is loaded with vector loads
    const int32_t* order;
    const int32_t* seg_first;
    const int32_t* seg_row;
    const int64_t* seg_lo;
    const int64_t* seg_hi;
    const int32_t* seg_order;  // processing order of the segments
    int32_t nseg;
    float* seg_part;
    int32_t* fb_list;
    int32_t* cursors;
    unsigned long long* counters;
    float tau;
    int32_t rows_batch;   // 0: static round-robin rows; 1: rows from the shared queue
    double* fb_scratch;   // float64 Hessians of the wide-block fallback (one B x B per workgroup)
    int32_t seg_len;      // segment length of long rows
    int32_t seg_group;    // a row's segment partials are summed in groups of this many (k_seg_group)
};

// One fold-in request as the fold-in kernel reads it (from device or pinned host memory).
struct FoldReq {
    const int32_t* items;  // [n] item ids
    const float* y;        // [n] labels (null: ones)
    float* ws;             // device scratch of fold_ws_floats(n) floats, 256-byte aligned
    float* out;            // [d] the folded-in row (device or pinned host memory)
    int32_t* st;           // per-request status bits (FOLD_ST_*), may be null
    int32_t n;
    int32_t copy;          // 1: items / y are first copied into ws (host-resident inputs)
};
enum FoldStatus : int { FOLD_ST_FLOAT64 = 1, FOLD_ST_NOT_SPD = 2, FOLD_ST_BAD_ID = 4 };
// Global fold-in counters (int32): bad ids, requests redone in float64, not SPD in float64.
enum FoldCounter : int { FOLD_CNT_BAD_ID = 0, FOLD_CNT_FLOAT64 = 1, FOLD_CNT_NOT_SPD = 2, FOLD_CNT_NUM = 4 };

// Launch shape of the fold-in kernel for one (item table, d, b).
struct FoldShape {
    int32_t I = 0, d = 0, b = 0, nb = 0, B = 0;
    bool gfac = false;     // the inverse factors live in ws instead of LDS
    int32_t nl = 0;        // requests of up to nl items keep ids and residuals in LDS
    size_t lds_bytes = 0;  // dynamic LDS per workgroup
};

}  // namespace ials

struct ials_ctx {
    // configuration
    int32_t U = 0, I = 0, d = 0, b = 0, B = 0;  // B = b padded to a multiple of 16
    float alpha0 = 0.f, lambda = 0.f, tau = 1e-4f;
    int32_t precision = 0;
    int32_t seg_len = ials::kSegLenDefault;
    int32_t gram_split = ials::kGramSplitDefault;  // workgroups the Gramian slab's split-K is sized for
    int64_t nnz = 0;
    hipStream_t stream = nullptr;
    int device = 0;
    int num_cu = 256;

    // borrowed
    float* W = nullptr;
    float* H = nullptr;

    // owned
    ials::SideIndex side[2];
    float* yhat = nullptr;       // [nnz] user-major: prediction minus the part of block cur_block
    int32_t cur_block = 0;       // the block the prediction cache is relative to
    float* pred = nullptr;       // [nnz] predictions materialised on request
    float* G = nullptr;          // [d * B] partial Gramian of the fixed side
    float* Dmat = nullptr;       // [B * B] alpha0 * G_pipi + lambda I (identity on padding)
    float* dtiles = nullptr;     // [B * B + ...] the same in the MFMA accumulator layout
    float* R0 = nullptr;         // [max(U,I) * B] dense gradient term
    float* gram_part = nullptr;  // split-K partials
    size_t gram_part_floats = 0;
    float* seg_part = nullptr;   // per-segment partial Hessian + gradient
    double* fb_scratch = nullptr;  // float64 fallback Hessians when B > 64
    int32_t* fb_list = nullptr;  // [max(U,I)]
    int32_t* cursors = nullptr;  // [CUR_NUM]
    unsigned long long* counters = nullptr;  // [CNT_NUM]
    double* loss_part = nullptr;  // loss partial sums
    size_t loss_part_len = 0;
    double* gram64 = nullptr;    // [2 * d * d] float64 Gramians for the loss
    double* loss_out = nullptr;  // [4]
    uint32_t flags = 0;
    bool own_stream = false;
    hipGraphExec_t epoch_exec = nullptr;  // captured epoch (IALS_FLAG_GRAPH)
    uint64_t device_bytes = 0;   // library-owned allocations held until destroy
    uint64_t tmp_bytes = 0;      // create-time temporaries held now
    uint64_t peak_bytes = 0;     // max of device_bytes + tmp_bytes so far
    uint64_t budget = 0;
    int64_t passes = 0;

    // fold-in of new rows against H (ials_foldin)
    ials::FoldShape fold;
    float* fold_G = nullptr;          // [d * d] H^T H
    int64_t fold_G_passes = -1;       // pass count when fold_G was formed
    float* fold_ws = nullptr;         // request scratch
    size_t fold_ws_cap = 0;           // floats
    ials::FoldReq* fold_req = nullptr;  // pinned host descriptors
    int32_t fold_req_cap = 0;
    int32_t* fold_cnt = nullptr;      // [FOLD_CNT_NUM] device counters
    int64_t fold_requests = 0, fold_float64 = 0;

    std::string err;
    std::vector<void*> owned;       // every device allocation of this context
    std::vector<void*> owned_host;  // pinned host allocations

    // per-kernel timing (HIP events on the stream), off by default
    bool prof = false;
    std::vector<hipEvent_t> prof_pool;   // 2 events per recorded launch
    std::vector<int> prof_kind;          // family of each recorded launch
    size_t prof_used = 0;
    double prof_ms[IALS_K_NUM] = {};
    int64_t prof_count[IALS_K_NUM] = {};
};

namespace ials {
// p += t * (lane J of this lane's 16-lane row of D): v_fmac_f32 with a DPP row_newbcast
// source operand.  The first update of a step begins with two wait states, as a DPP read
// of a VGPR that a VALU instruction has just written requires; the updates of one step are
// volatile so they keep their order and D is not rewritten between them.
template <int J, bool FIRST>
__device__ inline void fmac_rowbcast(float& p, float D, float t) {
    if constexpr (FIRST)
        asm volatile("s_nop 1\n\tv_fmac_f32_dpp %0, %1, %2 row_newbcast:%3 row_mask:0xf bank_mask:0xf bound_ctrl:1"
                     : "+v"(p)
                     : "v"(D), "v"(t), "i"(J));
    else
        asm volatile("v_fmac_f32_dpp %0, %1, %2 row_newbcast:%3 row_mask:0xf bank_mask:0xf bound_ctrl:1"
                     : "+v"(p)
                     : "v"(D), "v"(t), "i"(J));
}
// Columns JJ..15 of one elimination step: p[jj] += D(row lane jj) * t.
template <int JJ, bool FIRST>
__device__ inline void eliminate_cols(float* p, float D, float t) {
    if constexpr (JJ < 16) {
        fmac_rowbcast<JJ, FIRST>(p[JJ], D, t);
        eliminate_cols<JJ + 1, false>(p, D, t);
    }
}
}  // namespace ials

namespace ials {
// Brackets the launches issued in its lifetime with events when profiling is on.
struct ProfScope {
    ials_ctx* c;
    int kind;
    size_t slot = (size_t)-1;
    ProfScope(ials_ctx* c_, int kind_) : c(c_), kind(kind_) {
        if (c->prof && 2 * (c->prof_used + 1) <= c->prof_pool.size()) {
            slot = c->prof_used++;
            c->prof_kind[slot] = kind;
            (void)hipEventRecord(c->prof_pool[2 * slot], c->stream);
        }
    }
    ~ProfScope() {
        if (slot != (size_t)-1) (void)hipEventRecord(c->prof_pool[2 * slot + 1], c->stream);
    }
};
}  // namespace ials

namespace ials {

// Host-side launchers (implemented in the .hip files).
ials_status build_index(ials_ctx* c, const int32_t* d_user, const int32_t* d_item, const float* d_y,
                        const float* d_a);
void launch_predict(ials_ctx* c, int32_t blk, bool inside, float* out);
void launch_gramian_slab(ials_ctx* c, const float* X, int32_t n, int32_t p0, int32_t bw, int32_t ncols,
                         float* out, bool make_dmat);
void launch_dense(ials_ctx* c, const float* X, int32_t n, int32_t p0, int32_t bw);
void launch_sweep(ials_ctx* c, int side, int32_t blk);
// The pass for blocks wider than 64 coordinates (B = 128 or 256).
void launch_sweep_big(ials_ctx* c, SweepArgs& A, const SideIndex& s, int sd, bool trans);
ials_status launch_loss(ials_ctx* c);
size_t gram_part_floats_needed(int32_t n, int32_t d, int32_t ncols, bool bf16);
// out (d x ncols) = X^T X[:, p0:p0+bw] with the split-K partials in part (gram_part_floats_needed floats);
// bf16: bfloat16 operands on the matrix cores, float32 partials, float64 reduction.
// split: workgroups the split-K of the 64 x 64-tile kernels is sized for (64..2048).
void launch_gramian_raw(hipStream_t st, const float* X, int32_t n, int32_t d, int32_t p0, int32_t bw, int32_t ncols,
                        float* part, float* out, bool bf16, int32_t split = kGramSplitDefault);
FoldShape fold_shape(int32_t I, int32_t d, int32_t b);
size_t fold_ws_floats(const FoldShape& f, int64_t n);
// Fold-in of m requests (one workgroup each) against H (I x d) and G = H^T H (d x d).
hipError_t launch_foldin(hipStream_t st, const FoldShape& f, const float* H, const float* G, float alpha0,
                         float lambda, float tau, int32_t passes, const FoldReq* reqs, int32_t m, int32_t* counters);
size_t seg_part_floats_per_segment(int32_t B);
// Group sums of segment partials (stride floats each) when A.seg_group > 1.
void launch_seg_group(hipStream_t st, const SweepArgs& A, int32_t stride);
size_t big_fallback_doubles(int32_t B);
// Float64 redo of the rows a wide-block pass (B = 128 or 256) rejected (A.fb_scratch set).
void launch_fallback_big(ials_ctx* c, const SweepArgs& A);

// out[e] = sum over nchunks partials part[c][e] (count floats each), added in float64 in a fixed order.
void launch_gram_reduce(hipStream_t st, const float* part, int32_t nchunks, int64_t count, float* out);
// p[0 .. n) = v on the stream (a kernel, capturable in graphs).
void launch_fill(hipStream_t st, float* p, int64_t n, float v);
// One pass of the b = 1 specialisation (coordinate descent, Alg. 2) for coordinate blk.
void launch_icd_pass(ials_ctx* c, int sd, int32_t blk);

// Workgroups of one kernel resident per CU, kept per device: set_lds raises the kernel's
// dynamic-LDS limit to lds bytes first (the limit is a per-device attribute), then the
// occupancy for threads-wide workgroups with lds bytes is queried once per device and
// cached in cache (one static OccCache per kernel instantiation).  fallback if the query fails.
struct OccCache {
    static constexpr int kDevices = 64;
    std::atomic<int> v[kDevices] = {};
};
int resident_per_cu(OccCache& cache, const void* kernel, int threads, size_t lds, bool set_lds, int fallback);

// Allocation helper that tracks the context's byte count and budget.
hipError_t dev_alloc(ials_ctx* c, void** p, size_t bytes);
// Create-time temporaries: counted against the same budget while they are held
// (device_bytes + tmp_bytes never exceeds it), released by tmp_free.
hipError_t tmp_alloc(ials_ctx* c, void** p, size_t bytes);
void tmp_free(ials_ctx* c, void* p, size_t bytes);
// The pivot threshold the kernels compare with (min pivot < tau * largest diagonal entry):
// <= 0 selects 1e-4; >= 1 becomes the largest float, so that every row fails the test (with
// tau = 1 a row whose pivots all equal its largest diagonal entry would pass).
inline float effective_tau(float ratio) {
    if (!(ratio > 0.f)) return 1e-4f;
    return ratio >= 1.f ? 3.4e38f : ratio;
}
// IALS_E_NOMEM for an allocation failure or an exceeded budget, IALS_E_HIP otherwise.
inline ials_status alloc_status(hipError_t e) { return e == hipErrorOutOfMemory ? IALS_E_NOMEM : IALS_E_HIP; }

}  // namespace ials

#define IALS_ALLOC_TRY(c, expr)                                                        \
    do {                                                                               \
        hipError_t e_ = (expr);                                                        \
        if (e_ != hipSuccess) {                                                        \
            (c)->err = std::string(#expr " failed: ") + hipGetErrorString(e_);         \
            return ials::alloc_status(e_);                                             \
        }                                                                              \
    } while (0)

#define IALS_HIP_TRY(c, expr)                                                          \
    do {                                                                               \
        hipError_t e_ = (expr);                                                        \
        if (e_ != hipSuccess) {                                                        \
            (c)->err = std::string(#expr " failed: ") + hipGetErrorString(e_);         \
            return IALS_E_HIP;                                                         \
        }                                                                              \
    } while (0)
