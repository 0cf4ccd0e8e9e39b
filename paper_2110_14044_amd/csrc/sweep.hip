// The block pass of iALS++ (sec. 4, eq. 8-9, Alg. 3) on gfx950.
//
// For every row r of the side being updated (users, or items) and the block
// pi = [p0, p0+bw) padded to B = 16*NT columns:
//   T      = X_other[partners(r), pi]            gathered straight from the embedding table
//   Hess   = alpha0 G_pipi + lambda I + T^T diag(a) T   (MFMA f32 16x16x4, lower tiles only)
//   grad   = R0[r] + T^T (a (yhat - y))          (R0 = alpha0 x_r G^pi + lambda x_{r,pi}, precomputed)
//   delta  = Hess^-1 grad                         (blocked Cholesky on the accumulator tiles)
//   x_{r,pi} -= delta;  yhat_k -= <delta, T_k>   (the delta update of the prediction cache)
//
// One wavefront owns one row at a time and takes rows from a work queue in
// order of decreasing length, so rows of very different lengths share the GPU
// evenly.  Rows longer than kSegLen observations are split into segments:
// k_sweep_seg accumulates each segment's partial Hessian and gradient, the row
// kernel adds them in segment order (a fixed order, so results are bitwise
// reproducible), solves, and k_patch_seg patches yhat segment by segment.
// A row whose float32 Cholesky pivots fall below tau * (largest pivot), or are
// not positive, is redone from scratch in float64 by k_sweep_fallback.
//
// Column order.  The MFMA position p = 16 t + m (tile t, lane m of a 16-lane
// group) stands for block column colmap(p).  When the block lies fully inside
// the row and is vector-aligned (FULL), lane m loads the NT consecutive columns
// NT*m .. NT*m+NT-1 with one vector load, so colmap(p) = NT*m + t; otherwise
// colmap(p) = p.  The Hessian, gradient and step are all formed in p order,
// which is a symmetric permutation of the block: the solution is the same.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "ials_internal.h"

namespace ials {
namespace {

struct SweepArgs {
    const int64_t* ptr;
    const int32_t* col;
    const int32_t* slot;  // yhat position per observation (null: identity)
    const float* y;       // labels in this side's order (null: ones)
    const float* a;       // weights in this side's order (null: ones)
    float* X;             // side being updated, N x d
    const float* Xo;      // fixed side
    float* yhat;
    const float* R0;      // N x B
    const float* Dmat;    // B x B
    float* dtiles;        // the Hessian start in accumulator layout (NTL x 64 x 4)
    int32_t d, p0, bw, nrows;
    const int32_t* order;
    const int32_t* seg_first;
    const int32_t* seg_row;
    const int64_t* seg_lo;
    const int64_t* seg_hi;
    int32_t nseg;
    float* seg_part;
    float* delta;
    int32_t* fb_list;
    int32_t* cursors;
    unsigned long long* counters;
    float tau;
};

__device__ inline floatx4 mfma4(float a, float b, floatx4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
__device__ inline float readlane(float x, int l) {
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x), l));
}
// Order LDS accesses of one wavefront (LDS operations of a wave execute in order).
__device__ inline void wave_lds_fence() {
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
}
__device__ inline int queue_next(int32_t* cursor, int lane) {
    int it = 0;
    if (lane == 0) it = atomicAdd(cursor, 1);
    return __builtin_amdgcn_readfirstlane(it);
}

template <int NT>
constexpr int ntiles() { return NT * (NT + 1) / 2; }

// floats of one segment partial: NTL tiles x 64 lanes x 4 + B gradient entries
template <int NT>
constexpr int seg_stride() { return ntiles<NT>() * 256 + 16 * NT; }

template <int NT, bool FULL>
__host__ __device__ constexpr int colmap(int p) { return FULL ? NT * (p & 15) + (p >> 4) : p; }

// x[t] = X_other[i][p0 + colmap(16 t + q16)], 0 outside the block.
template <int NT, bool FULL>
__device__ inline void gather_row(const SweepArgs& A, int i, int q16, float* x) {
    const float* xr = A.Xo + (size_t)i * A.d + A.p0;
    if constexpr (FULL && NT == 4) {
        const float4 v = *reinterpret_cast<const float4*>(xr + 4 * q16);
        x[0] = v.x;
        x[1] = v.y;
        x[2] = v.z;
        x[3] = v.w;
    } else if constexpr (FULL && NT == 2) {
        const float2 v = *reinterpret_cast<const float2*>(xr + 2 * q16);
        x[0] = v.x;
        x[1] = v.y;
    } else if constexpr (FULL && NT == 1) {
        x[0] = xr[q16];
    } else {
#pragma unroll
        for (int t = 0; t < NT; ++t) {
            const int c = 16 * t + q16;
            const float v = xr[c < A.bw ? c : A.bw - 1];
            x[t] = (c < A.bw) ? v : 0.f;
        }
    }
}

// acc (lower tiles, MFMA D layout, p order) += T^T diag(a) T and gp[t] (position
// 16t+q16, this lane group's share) += T^T (a (yhat - y)) over observations [lo, hi).
template <int NT, bool FULL>
__device__ inline void accumulate(const SweepArgs& A, int64_t lo, int64_t hi, floatx4* acc, float* gp, int lane) {
    const int q16 = lane & 15, g4 = lane >> 4;
    for (int64_t c0 = lo; c0 < hi; c0 += 64) {
        const int64_t k = c0 + lane;
        const bool v = k < hi;
        int ci = 0;
        float res = 0.f, aw = 0.f;
        if (v) {
            ci = A.col[k];
            const int64_t s = A.slot ? (int64_t)A.slot[k] : k;
            const float ak = A.a ? A.a[k] : 1.f;
            const float yk = A.y ? A.y[k] : 1.f;
            res = ak * (A.yhat[s] - yk);
            aw = ak;
        }
        const int nsteps = ((int)std::min<int64_t>(64, hi - c0) + 3) >> 2;
        for (int st = 0; st < nsteps; st += 4) {
            const int nv = std::min(4, nsteps - st);
            float x[4][NT], r4[4], a4[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                if (u < nv) {
                    const int src = 4 * (st + u) + g4;
                    const int i = __shfl(ci, src);
                    r4[u] = __shfl(res, src);
                    a4[u] = __shfl(aw, src);
                    gather_row<NT, FULL>(A, i, q16, x[u]);
                }
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                if (u < nv) {
                    float xa[NT];
#pragma unroll
                    for (int t = 0; t < NT; ++t) {
                        gp[t] = fmaf(r4[u], x[u][t], gp[t]);
                        xa[t] = a4[u] * x[u][t];
                    }
                    int id = 0;
#pragma unroll
                    for (int ti = 0; ti < NT; ++ti)
#pragma unroll
                        for (int tj = 0; tj <= ti; ++tj) {
                            acc[id] = mfma4(xa[ti], x[u][tj], acc[id]);
                            ++id;
                        }
                }
            }
        }
    }
}

// yhat_k -= <delta, x_other[k, pi]> over observations [lo, hi); dl[t] = delta at position 16t + q16.
template <int NT, bool FULL>
__device__ inline void patch(const SweepArgs& A, int64_t lo, int64_t hi, const float* dl, int lane) {
    const int q16 = lane & 15, g4 = lane >> 4;
    for (int64_t c0 = lo; c0 < hi; c0 += 64) {
        const int64_t k = c0 + lane;
        const bool v = k < hi;
        const int ci = v ? A.col[k] : 0;
        const int si = v ? (A.slot ? A.slot[k] : (int)k) : 0;
        const int cnt = (int)std::min<int64_t>(64, hi - c0);
        const int nsteps = (cnt + 3) >> 2;
        for (int st = 0; st < nsteps; st += 4) {
            const int nv = std::min(4, nsteps - st);
            float x[4][NT];
            int sd[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                if (u < nv) {
                    const int src = 4 * (st + u) + g4;
                    const int i = __shfl(ci, src);
                    sd[u] = __shfl(si, src);
                    gather_row<NT, FULL>(A, i, q16, x[u]);
                }
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                if (u < nv) {
                    float dot = 0.f;
#pragma unroll
                    for (int t = 0; t < NT; ++t) dot = fmaf(x[u][t], dl[t], dot);
                    dot += __shfl_xor(dot, 8);
                    dot += __shfl_xor(dot, 4);
                    dot += __shfl_xor(dot, 2);
                    dot += __shfl_xor(dot, 1);
                    if (q16 == 0 && 4 * (st + u) + g4 < cnt) A.yhat[sd[u]] -= dot;
                }
            }
        }
    }
}

template <int NT, bool FULL>
__global__ __launch_bounds__(256) void k_sweep_seg(SweepArgs A) {
    constexpr int NTL = ntiles<NT>();
    const int lane = threadIdx.x & 63, q16 = lane & 15, g4 = lane >> 4;
    for (;;) {
        const int it = queue_next(&A.cursors[CUR_SEGS], lane);
        if (it >= A.nseg) break;
        floatx4 acc[NTL];
        float gp[NT];
#pragma unroll
        for (int id = 0; id < NTL; ++id) acc[id] = floatx4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int t = 0; t < NT; ++t) gp[t] = 0.f;
        accumulate<NT, FULL>(A, A.seg_lo[it], A.seg_hi[it], acc, gp, lane);
#pragma unroll
        for (int t = 0; t < NT; ++t) {
            gp[t] += __shfl_xor(gp[t], 16);
            gp[t] += __shfl_xor(gp[t], 32);
        }
        float* P = A.seg_part + (size_t)it * seg_stride<NT>();
#pragma unroll
        for (int id = 0; id < NTL; ++id) *reinterpret_cast<floatx4*>(P + ((size_t)id * 64 + lane) * 4) = acc[id];
        if (g4 == 0) {
#pragma unroll
            for (int t = 0; t < NT; ++t) P[NTL * 256 + 16 * t + q16] = gp[t];
        }
    }
}

// Blocked Cholesky storage: panel K (16 columns, rows 16K..B-1) of the factor L is
// kept in LDS with row stride kPS; panels are packed one after another.
constexpr int kPS = 16;
template <int NT>
constexpr int panel_rows() { return 16 * NT * (NT + 1) / 2; }
template <int NT>
__host__ __device__ constexpr int panel_row0(int K) { return 16 * (K * NT - K * (K - 1) / 2); }
// LDS floats of k_sweep_rows per wavefront: the packed panels and two 64-entry
// broadcast columns.
template <int NT>
constexpr int rows_lds_floats_per_wave() { return panel_rows<NT>() * kPS + 128; }
template <int NT>
constexpr int rows_lds_floats() { return 4 * rows_lds_floats_per_wave<NT>(); }

// alpha0 G_pipi + lambda I laid out as the accumulator tiles in p order (the start
// of every Hessian of the pass): dtiles[(id * 64 + lane) * 4 + j].
template <int NT, bool FULL>
__global__ void k_make_dtiles(const float* __restrict__ Dmat, float* __restrict__ dtiles) {
    constexpr int B = 16 * NT, NTL = ntiles<NT>();
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= NTL * 256) return;
    const int id = e >> 8, lq = (e >> 2) & 63, j = e & 3;
    int ti = 0;
    while ((ti + 1) * (ti + 2) / 2 <= id) ++ti;
    const int tj = id - ti * (ti + 1) / 2;
    dtiles[e] = Dmat[colmap<NT, FULL>(16 * ti + 4 * (lq >> 4) + j) * B + colmap<NT, FULL>(16 * tj + (lq & 15))];
}

template <int NT, bool FULL>
__global__ __launch_bounds__(256, 3) void k_sweep_rows(SweepArgs A) {
    constexpr int B = 16 * NT, NTL = ntiles<NT>();
    extern __shared__ float lds_all[];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, q16 = lane & 15, g4 = lane >> 4;
    float* pan = lds_all + wave * rows_lds_floats_per_wave<NT>();
    float* colA = pan + panel_rows<NT>() * kPS;
    float* colG = colA + 64;
    const int my_col = colmap<NT, FULL>(lane < B ? lane : 0);

    for (;;) {
        const int it = queue_next(&A.cursors[CUR_ROWS], lane);
        if (it >= A.nrows) break;
        const int r = A.order[it];
        const int64_t lo = A.ptr[r], hi = A.ptr[r + 1];
        floatx4 acc[NTL];
#pragma unroll
        for (int id = 0; id < NTL; ++id) acc[id] = *reinterpret_cast<const floatx4*>(A.dtiles + id * 256 + lane * 4);
        float gp[NT];
#pragma unroll
        for (int t = 0; t < NT; ++t) gp[t] = 0.f;
        const int sf = A.seg_first[r];
        if (sf < 0) {
            accumulate<NT, FULL>(A, lo, hi, acc, gp, lane);
#pragma unroll
            for (int t = 0; t < NT; ++t) {
                gp[t] += __shfl_xor(gp[t], 16);
                gp[t] += __shfl_xor(gp[t], 32);
            }
        } else {
            const int ns = (int)((hi - lo + kSegLen - 1) / kSegLen);
            for (int s = sf; s < sf + ns; ++s) {
                const float* P = A.seg_part + (size_t)s * seg_stride<NT>();
#pragma unroll
                for (int id = 0; id < NTL; ++id)
                    acc[id] += *reinterpret_cast<const floatx4*>(P + ((size_t)id * 64 + lane) * 4);
#pragma unroll
                for (int t = 0; t < NT; ++t) gp[t] += P[NTL * 256 + 16 * t + q16];
            }
        }
        // lane p < B holds the gradient entry of position p
        float g = 0.f;
#pragma unroll
        for (int t = 0; t < NT; ++t)
            if (g4 == t) g = gp[t];
        if (lane < B) g += A.R0[(size_t)r * B + my_col];

        // The lane id is laundered once per row so that lane-vs-k masks below are
        // formed inside the row, not hoisted out of the row loop into scalar registers.
        int ln = lane;
        asm volatile("" : "+v"(ln));

        // Blocked right-looking Cholesky on the accumulator tiles, 16 columns per panel,
        // with the forward substitution folded in.  Inside a panel, step k publishes
        // every row's column-k entry and gradient entry; with piv = A_kk and
        // t_i = A_ik / piv for rows i > k (0 otherwise), A_ij -= t_i A_jk for the
        // panel's later columns j and g_i -= t_i g_k; A_ik is then scaled to L_ik.
        // The finished panel updates the trailing tiles on the matrix cores.
#pragma unroll
        for (int K = 0; K < NT; ++K) {
            float* PK = pan + panel_row0<NT>(K) * kPS;  // row r >= 16K at PK + (r - 16K) * kPS
#pragma unroll
            for (int I = K; I < NT; ++I) {
                const int id = I * (I + 1) / 2 + K;
#pragma unroll
                for (int j = 0; j < 4; ++j) PK[(16 * (I - K) + 4 * g4 + j) * kPS + q16] = acc[id][j];
            }
            wave_lds_fence();
            const bool mine = (ln >= 16 * K) && (ln < B);
            const int prow = mine ? ln - 16 * K : 0;
            float p[16];
#pragma unroll
            for (int c4 = 0; c4 < 4; ++c4) {
                const float4 v = *reinterpret_cast<const float4*>(PK + prow * kPS + 4 * c4);
                p[4 * c4 + 0] = mine ? v.x : 0.f;
                p[4 * c4 + 1] = mine ? v.y : 0.f;
                p[4 * c4 + 2] = mine ? v.z : 0.f;
                p[4 * c4 + 3] = mine ? v.w : 0.f;
            }
#pragma unroll
            for (int c = 0; c < 16; ++c)
                if (16 * K + c > ln) p[c] = 0.f;
            wave_lds_fence();
#pragma unroll
            for (int kk = 0; kk < 16; ++kk) {
                const int k = 16 * K + kk;
                colA[lane] = p[kk];
                colG[lane] = g;
                wave_lds_fence();
                const float piv = colA[k];
                const float gk = colG[k];
                const float rs = (piv > 0.f) ? __builtin_amdgcn_rsqf(piv) : 0.f;
                const float t = (ln > k) ? p[kk] * (rs * rs) : 0.f;
                g = fmaf(-t, gk, g);
#pragma unroll
                for (int j4 = (kk + 1) / 4; j4 < 4; ++j4) {
                    const float4 c = *reinterpret_cast<const float4*>(colA + 16 * K + 4 * j4);
                    if (4 * j4 + 0 > kk) p[4 * j4 + 0] = fmaf(-t, c.x, p[4 * j4 + 0]);
                    if (4 * j4 + 1 > kk) p[4 * j4 + 1] = fmaf(-t, c.y, p[4 * j4 + 1]);
                    if (4 * j4 + 2 > kk) p[4 * j4 + 2] = fmaf(-t, c.z, p[4 * j4 + 2]);
                    if (4 * j4 + 3 > kk) p[4 * j4 + 3] = fmaf(-t, c.w, p[4 * j4 + 3]);
                }
                p[kk] *= rs;
                wave_lds_fence();
                __builtin_amdgcn_sched_barrier(0);
            }
            if (mine) {
#pragma unroll
                for (int c4 = 0; c4 < 4; ++c4)
                    *reinterpret_cast<float4*>(PK + prow * kPS + 4 * c4) =
                        make_float4(p[4 * c4], p[4 * c4 + 1], p[4 * c4 + 2], p[4 * c4 + 3]);
            }
            wave_lds_fence();
            // trailing tiles: A_IJ -= L_IK L_JK^T for K < J <= I
            if (K + 1 < NT) {
#pragma unroll
                for (int s4 = 0; s4 < 4; ++s4) {
                    float op[NT];
#pragma unroll
                    for (int I = K + 1; I < NT; ++I) op[I] = PK[(16 * (I - K) + q16) * kPS + 4 * s4 + g4];
#pragma unroll
                    for (int I = K + 1; I < NT; ++I)
#pragma unroll
                        for (int J = K + 1; J <= I; ++J) {
                            const int id = I * (I + 1) / 2 + J;
                            acc[id] = mfma4(-op[I], op[J], acc[id]);
                        }
                }
            }
            __builtin_amdgcn_sched_barrier(0);
        }
        // diagonal of L for this lane's row, from the panel that holds it
        const int pk = ln >> 4;
        const int pbase = panel_row0<NT>(pk) - 16 * pk;
        const float lii = pan[(ln < B ? pbase + ln : 0) * kPS + (ln & 15)];
        const float dinv = (ln < B && lii > 0.f) ? 1.f / lii : 0.f;
        const float mypiv = lii * lii;
        // pivot check over the real (unpadded) coordinates
        const bool real = (ln < B) && (my_col < A.bw);
        float pmin = real ? mypiv : 3.0e38f;
        float pmax = real ? mypiv : 0.f;
#pragma unroll
        for (int m = 1; m < 64; m <<= 1) {
            pmin = fminf(pmin, __shfl_xor(pmin, m));
            pmax = fmaxf(pmax, __shfl_xor(pmax, m));
        }
        const bool bad = !(pmin > 0.f) || (pmin < A.tau * pmax);
        if (bad) {
            if (lane == 0) {
                const int pos = atomicAdd(&A.cursors[CUR_FB_LIST], 1);
                A.fb_list[pos] = r;
            }
            if (sf >= 0 && lane < B) A.delta[(size_t)r * B + lane] = 0.f;
            continue;
        }
        g *= dinv;  // y = L^-1 grad
        // Back substitution L^T x = y, 16 rows of L at a time from the last band;
        // lane i reads L[k][i] of the band from the panel that holds column i.
        const float gdinv = dinv;
#pragma unroll
        for (int K = NT - 1; K >= 0; --K) {
            float lt[16];
#pragma unroll
            for (int jj = 0; jj < 16; ++jj) {
                const bool ok = (pk <= K) && (ln <= 16 * K + jj) && (ln < B);
                const int rowi = ok ? pbase + 16 * K + jj : 0;
                const float v = pan[rowi * kPS + (ln & 15)];
                lt[jj] = ok ? v : 0.f;
            }
#pragma unroll
            for (int jj = 15; jj >= 0; --jj) {
                const int k = 16 * K + jj;
                const float xk = readlane(g * gdinv, k);
                g = (ln == k) ? xk : ((ln < k) ? fmaf(-lt[jj], xk, g) : g);
            }
            __builtin_amdgcn_sched_barrier(0);
        }
        wave_lds_fence();
        // g (lane p) = delta at block column colmap(p)
        if (lane < B && my_col < A.bw) A.X[(size_t)r * A.d + A.p0 + my_col] -= g;
        if (sf >= 0) {
            if (lane < B) A.delta[(size_t)r * B + lane] = g;
            continue;
        }
        float dl[NT];
#pragma unroll
        for (int t = 0; t < NT; ++t) dl[t] = __shfl(g, 16 * t + q16);
        patch<NT, FULL>(A, lo, hi, dl, lane);
    }
}

template <int NT, bool FULL>
__global__ __launch_bounds__(256) void k_patch_seg(SweepArgs A) {
    constexpr int B = 16 * NT;
    const int lane = threadIdx.x & 63, q16 = lane & 15;
    for (;;) {
        const int it = queue_next(&A.cursors[CUR_PATCH], lane);
        if (it >= A.nseg) break;
        const int r = A.seg_row[it];
        float dl[NT];
#pragma unroll
        for (int t = 0; t < NT; ++t) dl[t] = A.delta[(size_t)r * B + 16 * t + q16];
        patch<NT, FULL>(A, A.seg_lo[it], A.seg_hi[it], dl, lane);
    }
}

// Float64 redo of rows whose float32 factorisation was rejected: the Hessian and
// gradient are re-accumulated from the gathered rows in float64, factored and
// solved in float64; the row is then updated and (short rows) its yhat patched.
template <int NT, bool FULL>
__global__ __launch_bounds__(256) void k_sweep_fallback(SweepArgs A) {
    constexpr int B = 16 * NT;
    constexpr int CH = 32;
    __shared__ double Hm[B][B + 1];
    __shared__ double xs[CH][B];
    __shared__ double gv[B];
    __shared__ double rs[CH], ws[CH];
    __shared__ int ok;
    const int tid = threadIdx.x;
    const int nfb = A.cursors[CUR_FB_LIST];
    for (int idx = blockIdx.x; idx < nfb; idx += gridDim.x) {
        const int r = A.fb_list[idx];
        const int64_t lo = A.ptr[r], hi = A.ptr[r + 1];
        for (int e = tid; e < B * B; e += 256) Hm[e / B][e % B] = (double)A.Dmat[e];
        if (tid < B) gv[tid] = (double)A.R0[(size_t)r * B + tid];
        if (tid == 0) ok = 1;
        __syncthreads();
        for (int64_t c0 = lo; c0 < hi; c0 += CH) {
            for (int e = tid; e < CH * B; e += 256) {
                const int j = e / B, c = e % B;
                const int64_t k = c0 + j;
                xs[j][c] = (k < hi && c < A.bw) ? (double)A.Xo[(size_t)A.col[k] * A.d + A.p0 + c] : 0.0;
            }
            if (tid < CH) {
                const int64_t k = c0 + tid;
                double res = 0.0, w = 0.0;
                if (k < hi) {
                    const int64_t s = A.slot ? (int64_t)A.slot[k] : k;
                    const double ak = A.a ? (double)A.a[k] : 1.0;
                    const double yk = A.y ? (double)A.y[k] : 1.0;
                    res = ak * ((double)A.yhat[s] - yk);
                    w = ak;
                }
                rs[tid] = res;
                ws[tid] = w;
            }
            __syncthreads();
            for (int e = tid; e < B * B; e += 256) {
                const int p = e / B, q = e % B;
                double s = 0.0;
                for (int j = 0; j < CH; ++j) s += ws[j] * xs[j][p] * xs[j][q];
                Hm[p][q] += s;
            }
            if (tid < B) {
                double s = 0.0;
                for (int j = 0; j < CH; ++j) s += rs[j] * xs[j][tid];
                gv[tid] += s;
            }
            __syncthreads();
        }
        // Cholesky in float64 (lower triangle)
        for (int k = 0; k < B; ++k) {
            if (tid == 0) {
                const double piv = Hm[k][k];
                if (!(piv > 0.0)) ok = 0;
                Hm[k][k] = piv > 0.0 ? sqrt(piv) : 1.0;
            }
            __syncthreads();
            for (int i = k + 1 + tid; i < B; i += 256) Hm[i][k] /= Hm[k][k];
            __syncthreads();
            for (int e = tid; e < B * B; e += 256) {
                const int i = e / B, j = e % B;
                if (j > k && i >= j) Hm[i][j] -= Hm[i][k] * Hm[j][k];
            }
            __syncthreads();
        }
        if (tid == 0) {
            for (int i = 0; i < B; ++i) {
                double t = gv[i];
                for (int k = 0; k < i; ++k) t -= Hm[i][k] * gv[k];
                gv[i] = t / Hm[i][i];
            }
            for (int i = B - 1; i >= 0; --i) {
                double t = gv[i];
                for (int k = i + 1; k < B; ++k) t -= Hm[k][i] * gv[k];
                gv[i] = t / Hm[i][i];
            }
            if (!ok) {
                atomicAdd(&A.counters[CNT_NOT_SPD], 1ull);
                for (int i = 0; i < B; ++i) gv[i] = 0.0;
            }
            atomicAdd(&A.counters[CNT_FALLBACK_ROWS], 1ull);
        }
        __syncthreads();
        if (tid < A.bw) A.X[(size_t)r * A.d + A.p0 + tid] -= (float)gv[tid];
        if (A.seg_first[r] >= 0) {
            if (tid < B) A.delta[(size_t)r * B + tid] = (float)gv[colmap<NT, FULL>(tid)];
        } else {
            for (int64_t k = lo + tid; k < hi; k += 256) {
                const float* xr = A.Xo + (size_t)A.col[k] * A.d + A.p0;
                double dot = 0.0;
                for (int c = 0; c < A.bw; ++c) dot += gv[c] * (double)xr[c];
                const int64_t s = A.slot ? (int64_t)A.slot[k] : k;
                A.yhat[s] -= (float)dot;
            }
        }
        __syncthreads();
    }
}

template <int NT, bool FULL>
void launch_sweep_nt(ials_ctx* c, const SweepArgs& args, const SideIndex& s, int sd) {
    hipStream_t st = c->stream;
    const unsigned max_blocks = (unsigned)c->num_cu * 8;
    if (s.nseg > 0) {
        ProfScope ps(c, IALS_K_SEG_USER + sd);
        hipLaunchKernelGGL((k_sweep_seg<NT, FULL>), dim3(std::min<unsigned>(max_blocks, (s.nseg + 3) / 4)), dim3(256),
                           0, st, args);
    }
    if (s.nrows > 0) {
        const size_t lds = sizeof(float) * rows_lds_floats<NT>();
        hipLaunchKernelGGL((k_make_dtiles<NT, FULL>), dim3((ntiles<NT>() * 256 + 255) / 256), dim3(256), 0, st, args.Dmat,
                           args.dtiles);
        {
            ProfScope ps(c, IALS_K_ROWS_USER + sd);
            hipLaunchKernelGGL((k_sweep_rows<NT, FULL>), dim3(std::min<unsigned>(max_blocks, (s.nrows + 3) / 4)),
                               dim3(256), lds, st, args);
        }
        ProfScope ps(c, IALS_K_FALLBACK_USER + sd);
        hipLaunchKernelGGL((k_sweep_fallback<NT, FULL>), dim3((unsigned)c->num_cu), dim3(256), 0, st, args);
    }
    if (s.nseg > 0) {
        ProfScope ps(c, IALS_K_PATCH_USER + sd);
        hipLaunchKernelGGL((k_patch_seg<NT, FULL>), dim3(std::min<unsigned>(max_blocks, (s.nseg + 3) / 4)), dim3(256),
                           0, st, args);
    }
}

template <int NT>
void launch_sweep_full_or_not(ials_ctx* c, const SweepArgs& A, const SideIndex& s, int sd) {
    constexpr int B = 16 * NT;
    const int vec = (NT == 3) ? 0 : NT;
    bool full = vec > 0 && A.bw == B && (A.d % vec == 0) && (A.p0 % vec == 0) &&
                ((reinterpret_cast<uintptr_t>(A.Xo) % (4 * vec)) == 0);
    if constexpr (NT == 3) full = false;
    if (full)
        launch_sweep_nt<NT, true>(c, A, s, sd);
    else
        launch_sweep_nt<NT, false>(c, A, s, sd);
}

}  // namespace

size_t seg_part_floats_per_segment(int32_t B) {
    const int NT = B / 16;
    return (size_t)(NT * (NT + 1) / 2) * 256 + (size_t)B;
}

void launch_sweep(ials_ctx* c, int sd, int32_t p0, int32_t bw) {
    const SideIndex& s = c->side[sd];
    SweepArgs A;
    A.ptr = s.ptr;
    A.col = s.col;
    A.slot = s.slot;
    A.y = s.y;
    A.a = s.a;
    A.X = sd == IALS_SIDE_USER ? c->W : c->H;
    A.Xo = sd == IALS_SIDE_USER ? c->H : c->W;
    A.yhat = c->yhat;
    A.R0 = c->R0;
    A.Dmat = c->Dmat;
    A.dtiles = c->dtiles;
    A.d = c->d;
    A.p0 = p0;
    A.bw = bw;
    A.nrows = s.nrows;
    A.order = s.order;
    A.seg_first = s.seg_first;
    A.seg_row = s.seg_row;
    A.seg_lo = s.seg_lo;
    A.seg_hi = s.seg_hi;
    A.nseg = s.nseg;
    A.seg_part = c->seg_part;
    A.delta = c->delta;
    A.fb_list = c->fb_list;
    A.cursors = c->cursors;
    A.counters = c->counters;
    A.tau = c->tau;
    switch (c->B) {
        case 16: launch_sweep_full_or_not<1>(c, A, s, sd); break;
        case 32: launch_sweep_full_or_not<2>(c, A, s, sd); break;
        case 48: launch_sweep_full_or_not<3>(c, A, s, sd); break;
        default: launch_sweep_full_or_not<4>(c, A, s, sd); break;
    }
}

}  // namespace ials
