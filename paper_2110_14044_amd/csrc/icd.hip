// The b = 1 end of the block sweep: coordinate descent (iCD, Alg. 2), one coordinate f of
// one side per pass, without the padded 16-wide block machinery.
//
// Per pass (side with table X, partner table Xo, coordinate f):
//   k_icd_gcol   column f of the partner's Gramian, g = Xo^T Xo[:, f] (d floats; Alg. 2's
//                g^I), as row-chunk partials reduced in float64 by k_gram_reduce; the same
//                sweep over Xo copies the partner column Xo[:, f] (and, when the pass moves
//                the prediction cache, the column the cache was relative to) into contiguous
//                vectors, so that the per-observation gathers below read 4 bytes from a
//                vector that stays in the L2 instead of one float of a d-float row
//   k_icd_seg    rows longer than the segment length: one wavefront per segment sums
//                alpha (yhat - y) o_f and alpha o_f^2 over its observations (partials)
//   k_icd_rows   one wavefront per row: the same sums over the row's observations (or its
//                segments' partials in order), the dense term alpha0 <x_r, g> + lambda x_rf
//                (Alg. 2's gradient start), the scalar Newton step delta = grad / hess
//                (hess = alpha0 g_f + lambda + sum alpha o_f^2) and x_rf -= delta.
//
// The prediction cache is kept relative to the current coordinate (the b = 1 case of the
// block-relative cache): c = yhat - x_f o_f, so the residual of an observation is
// c + x_f o_f - y and no per-observation patch follows an update; the first user pass of a
// new coordinate moves the cache, c' = c + x_p o_p - x_f o_f.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>

#include "ials_internal.h"

namespace ials {
namespace {

inline unsigned nblk(int64_t n, int t) { return (unsigned)((n + t - 1) / t); }

__device__ inline float wave_sum(float s) {
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) s += __shfl_xor(s, m);
    return s;
}

// part[chunk][e] = sum over the chunk's rows r of Xo[r][e] Xo[r][f] (e in this block's 256
// columns); colf[r] = Xo[r][f] and, if colp, colp[r] = Xo[r][pc].  Rows are read eight at a
// time so that eight loads per thread are in flight.
__global__ __launch_bounds__(256) void k_icd_gcol(int32_t n, int32_t d, const float* __restrict__ Xo, int32_t f,
                                                  int32_t pc, int32_t rows_per_chunk, float* __restrict__ part,
                                                  float* __restrict__ colf, float* __restrict__ colp) {
    const int e = blockIdx.x * 256 + threadIdx.x;
    const bool on = e < d;
    const int ec = on ? e : 0;
    const int64_t r0 = (int64_t)blockIdx.y * rows_per_chunk;
    const int64_t r1 = std::min<int64_t>(n, r0 + rows_per_chunk);
    const bool wf = on && e == f, wp = on && colp != nullptr && e == pc;
    float acc = 0.f;
    int64_t r = r0;
    for (; r + 8 <= r1; r += 8) {
        float v[8], s[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            v[j] = Xo[(size_t)(r + j) * d + ec];
            s[j] = Xo[(size_t)(r + j) * d + f];
        }
#pragma unroll
        for (int j = 0; j < 8; ++j) acc = fmaf(v[j], s[j], acc);
        if (wf)
#pragma unroll
            for (int j = 0; j < 8; ++j) colf[r + j] = v[j];
        if (wp)
#pragma unroll
            for (int j = 0; j < 8; ++j) colp[r + j] = v[j];
    }
    for (; r < r1; ++r) {
        const float v = Xo[(size_t)r * d + ec];
        acc = fmaf(v, Xo[(size_t)r * d + f], acc);
        if (wf) colf[r] = v;
        if (wp) colp[r] = v;
    }
    if (on) part[(size_t)blockIdx.y * d + e] = acc;
}

struct IcdArgs {
    const int64_t* ptr;
    const int32_t* col;
    const int32_t* slot;  // cache position per observation (null: identity)
    const float* y;
    const float* a;
    float* X;             // this side, N x d
    float* cache;         // user-major prediction cache, relative to coordinate pc on entry
    const float* colf;    // partner column f
    const float* colp;    // partner column pc (moving pass only)
    const float* g;       // Gramian column f of the partner side (d floats)
    const int32_t* order;
    const int32_t* seg_first;
    const int32_t* seg_row;
    const int64_t* seg_lo;
    const int64_t* seg_hi;
    float* seg_part;      // 2 floats per segment: sum alpha r o_f, sum alpha o_f^2
    unsigned long long* counters;
    int32_t d, f, pc, nrows, nseg, seg_len;
    float alpha0, lambda;
};

// Sums over observations [lo, hi) of one row with own coordinates xf (and xp, the cache's
// coordinate, when TRANS): the cache moves to f on the way.
template <bool TRANS>
__device__ inline void icd_obs(const IcdArgs& A, int64_t lo, int64_t hi, float xf, float xp, int lane, float& sg,
                               float& sh) {
    for (int64_t k0 = lo; k0 < hi; k0 += 64) {
        const int64_t k = k0 + lane;
        if (k < hi) {
            const int j = A.col[k];
            const int64_t s = A.slot ? (int64_t)A.slot[k] : k;
            const float of = A.colf[j];
            const float ak = A.a ? A.a[k] : 1.f;
            const float yk = A.y ? A.y[k] : 1.f;
            float c = A.cache[s];
            if constexpr (TRANS) {
                c = fmaf(xp, A.colp[j], c);  // the prediction itself
                const float res = c - yk;
                A.cache[s] = fmaf(-xf, of, c);
                sg = fmaf(ak * res, of, sg);
            } else {
                const float res = fmaf(xf, of, c) - yk;
                sg = fmaf(ak * res, of, sg);
            }
            sh = fmaf(ak * of, of, sh);
        }
    }
}

template <bool TRANS>
__global__ __launch_bounds__(256) void k_icd_seg(IcdArgs A) {
    const int lane = threadIdx.x & 63;
    // uniform wavefront index: the segment index and its bounds are scalar
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    for (int sidx = blockIdx.x * 4 + wave; sidx < A.nseg; sidx += gridDim.x * 4) {
        const int r = A.seg_row[sidx];
        const float xf = A.X[(size_t)r * A.d + A.f];
        const float xp = TRANS ? A.X[(size_t)r * A.d + A.pc] : 0.f;
        float sg = 0.f, sh = 0.f;
        icd_obs<TRANS>(A, A.seg_lo[sidx], A.seg_hi[sidx], xf, xp, lane, sg, sh);
        sg = wave_sum(sg);
        sh = wave_sum(sh);
        if (lane == 0) {
            A.seg_part[2 * (size_t)sidx] = sg;
            A.seg_part[2 * (size_t)sidx + 1] = sh;
        }
    }
}

template <bool TRANS>
__global__ __launch_bounds__(256) void k_icd_rows(IcdArgs A) {
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    for (int it = blockIdx.x * 4 + wave; it < A.nrows; it += gridDim.x * 4) {
        const int r = A.order[it];
        float* xr = A.X + (size_t)r * A.d;
        const float xf = xr[A.f];
        const float xp = TRANS ? xr[A.pc] : 0.f;
        // dense term alpha0 <x_r, g> (the full current row, Alg. 2)
        float dot = 0.f;
        for (int e = lane; e < A.d; e += 64) dot = fmaf(xr[e], A.g[e], dot);
        float sg = 0.f, sh = 0.f;
        const int sf = A.seg_first[r];
        const int64_t lo = A.ptr[r], hi = A.ptr[r + 1];
        if (sf < 0) {
            icd_obs<TRANS>(A, lo, hi, xf, xp, lane, sg, sh);
        } else if (lane == 0) {
            // partials of the row's segments, added in segment order
            const int ns = (int)((hi - lo + A.seg_len - 1) / A.seg_len);
            for (int s = sf; s < sf + ns; ++s) {
                sg += A.seg_part[2 * (size_t)s];
                sh += A.seg_part[2 * (size_t)s + 1];
            }
        }
        dot = wave_sum(dot);
        sg = wave_sum(sg);
        sh = wave_sum(sh);
        if (lane == 0) {
            const float grad = fmaf(A.alpha0, dot, A.lambda * xf) + sg;
            const float hess = fmaf(A.alpha0, A.g[A.f], A.lambda) + sh;
            if (hess > 0.f) {
                xr[A.f] = xf - grad / hess;
            } else {
                // not positive even for this 1 x 1 "factorisation" (non-finite inputs): no step
                atomicAdd(&A.counters[CNT_NOT_SPD], 1ull);
                atomicAdd(&A.counters[CNT_FALLBACK_ROWS], 1ull);
            }
        }
    }
}

}  // namespace

// One iCD pass of coordinate blk on side sd (the cache moves to blk if it is relative to
// another coordinate).
void launch_icd_pass(ials_ctx* c, int sd, int32_t blk) {
    const SideIndex& s = c->side[sd];
    const bool user = sd == IALS_SIDE_USER;
    const float* Xo = user ? c->H : c->W;
    const int32_t no = user ? c->I : c->U;
    const int32_t d = c->d, f = blk, pc = c->cur_block;
    const bool trans = f != pc;
    hipStream_t st = c->stream;
    const int64_t nmax = std::max<int64_t>(c->U, c->I);
    float* colf = c->R0;
    float* colp = c->R0 + nmax;
    {
        ProfScope ps(c, IALS_K_GRAM_USER + sd);
        const unsigned cg = nblk(d, 256);
        // row chunks: about 2048 workgroups, within the split-K scratch
        int64_t chunks = std::max<int64_t>(1, 2048 / (int64_t)cg);
        chunks = std::min<int64_t>(chunks, std::max<int64_t>(1, (int64_t)(c->gram_part_floats / (size_t)d)));
        chunks = std::min<int64_t>(chunks, std::max<int64_t>(1, no));
        const int64_t rows = std::max<int64_t>(1, (no + chunks - 1) / chunks);
        chunks = std::max<int64_t>(1, (no + rows - 1) / rows);
        hipLaunchKernelGGL(k_icd_gcol, dim3(cg, (unsigned)chunks), dim3(256), 0, st, no, d, Xo, f, pc, (int32_t)rows,
                           c->gram_part, colf, trans ? colp : nullptr);
        launch_gram_reduce(st, c->gram_part, (int32_t)chunks, d, c->G);
    }
    IcdArgs A;
    A.ptr = s.ptr;
    A.col = s.col;
    A.slot = s.slot;
    A.y = s.y;
    A.a = s.a;
    A.X = user ? c->W : c->H;
    A.cache = c->yhat;
    A.colf = colf;
    A.colp = colp;
    A.g = c->G;
    A.order = s.order;
    A.seg_first = s.seg_first;
    A.seg_row = s.seg_row;
    A.seg_lo = s.seg_lo;
    A.seg_hi = s.seg_hi;
    A.seg_part = c->seg_part;
    A.counters = c->counters;
    A.d = d;
    A.f = f;
    A.pc = pc;
    A.nrows = s.nrows;
    A.nseg = s.nseg;
    A.seg_len = c->seg_len;
    A.alpha0 = c->alpha0;
    A.lambda = c->lambda;
    const unsigned max_blocks = (unsigned)c->num_cu * 16;
    if (s.nseg > 0) {
        ProfScope ps(c, IALS_K_SEG_USER + sd);
        if (trans)
            hipLaunchKernelGGL(k_icd_seg<true>, dim3(std::min<unsigned>(max_blocks, nblk(s.nseg, 4))), dim3(256), 0, st, A);
        else
            hipLaunchKernelGGL(k_icd_seg<false>, dim3(std::min<unsigned>(max_blocks, nblk(s.nseg, 4))), dim3(256), 0, st, A);
    }
    if (s.nrows > 0) {
        ProfScope ps(c, (trans ? IALS_K_ROWS_USER_MOVE : IALS_K_ROWS_USER) + sd);
        if (trans)
            hipLaunchKernelGGL(k_icd_rows<true>, dim3(std::min<unsigned>(max_blocks, nblk(s.nrows, 4))), dim3(256), 0, st, A);
        else
            hipLaunchKernelGGL(k_icd_rows<false>, dim3(std::min<unsigned>(max_blocks, nblk(s.nrows, 4))), dim3(256), 0, st, A);
    }
    c->cur_block = blk;
}

}  // namespace ials
