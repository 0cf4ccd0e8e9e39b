// Fold-in of new rows against a fixed item table (sec. 4, Alg. 3 applied to a
// single row whose partner side H never changes; eq. 3 is the limit it
// converges to).
//
// A request is a new user with observed items i_1..i_n (labels y, weights 1).
// Starting from w = 0 (so every prediction is 0), each of `passes` sweeps visits
// the blocks pi = [p0, p0+bw) in ascending order and takes the exact block step
//   grad  = alpha0 (w G)[pi] + lambda w[pi] + sum_k (yhat_k - y_k) h_{i_k}[pi]
//   Hess  = alpha0 G[pi,pi] + lambda I + sum_k h_{i_k}[pi] h_{i_k}[pi]^T
//   w[pi] -= Hess^-1 grad,   yhat_k -= <delta, h_{i_k}[pi]>
// with G = H^T H.  H is fixed, so every block's Hessian is the same in every
// sweep: it is accumulated on the matrix cores and Cholesky-factored once per
// request, and each block step is then a gradient, two triangular solves and
// the updates.
//
// One workgroup (4 wavefronts) per request.  Phase 1: the waves factor blocks
// in parallel (wave v takes blocks v, v+4, ...), keeping the factors in LDS
// (or in the request's scratch when they do not fit).  Phase 2: the block
// steps in order; the observed part of the gradient, the update of alpha0 w G
// and of the predictions are spread over the workgroup, the solve runs on one
// wavefront.  A request whose float32 pivots fail the ratio test is redone in
// float64 from scratch by the whole workgroup (the same iteration, with each
// block's Hessian rebuilt, factored and solved in float64).
#include <hip/hip_runtime.h>

#include <algorithm>

#include "ials_internal.h"

namespace ials {
namespace {

struct FoldArgs {
    const float* H;  // I x d
    const float* G;  // d x d
    int32_t I, d, b, nb;
    float alpha0, lambda, tau;
    int32_t passes;
    int32_t m;
    const FoldReq* req;
    int32_t* cnt;  // FOLD_CNT_NUM counters (may be null)
};

__device__ inline floatx4 mfma4(float a, float b, floatx4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
__device__ inline float readlane(float x, int l) {
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x), l));
}
__device__ inline void wave_fence() {
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
    __builtin_amdgcn_wave_barrier();
}
__device__ inline int item_at(const int32_t* items, int k, int I) {
    const int it = items[k];
    return (unsigned)it < (unsigned)I ? it : 0;  // ids are checked in phase 0; clamp keeps loads in bounds
}

// Scratch layout of one request (floats): predictions as n doubles, the item
// ids, the labels, then (global-factor mode) the factors.
__host__ __device__ inline size_t ws_items_off(int64_t n) { return (size_t)2 * n; }
__host__ __device__ inline size_t ws_y_off(int64_t n) { return (size_t)3 * n; }
__host__ __device__ inline size_t ws_fac_off(int64_t n) { return ((size_t)4 * n + 63) / 64 * 64; }

// Whole-workgroup float64 redo of one request (rare: only when the float32
// factorisation of some block fails the pivot test).
template <int B>
__device__ void foldin_f64(const FoldArgs& A, const FoldReq& R, int n, const int32_t* items, const float* yv,
                           double* sm, int* nspd) {
    const int tid = threadIdx.x, d = A.d, dp = (d + 3) & ~3;
    double* Am = sm;          // B x B
    double* w = Am + B * B;   // dp
    double* g = w + dp;       // B
    double* x = g + B;        // B
    double* yh = reinterpret_cast<double*>(R.ws);
    for (int f = tid; f < dp; f += 256) w[f] = 0.0;
    for (int k = tid; k < n; k += 256) yh[k] = 0.0;
    __syncthreads();
    for (int pass = 0; pass < A.passes; ++pass) {
        for (int blk = 0; blk < A.nb; ++blk) {
            const int p0 = blk * A.b, bw = min(A.b, d - p0);
            for (int e = tid; e < B * B; e += 256) {
                const int p = e / B, q = e % B;
                Am[e] = (p < bw && q < bw) ? (double)A.alpha0 * (double)A.G[(size_t)(p0 + p) * d + p0 + q] +
                                                 (p == q ? (double)A.lambda : 0.0)
                                           : (p == q ? 1.0 : 0.0);
            }
            if (tid < bw) {
                double s = 0.0;
                for (int f = 0; f < d; ++f) s += w[f] * (double)A.G[(size_t)f * d + p0 + tid];
                g[tid] = (double)A.alpha0 * s + (double)A.lambda * w[p0 + tid];
            }
            __syncthreads();
            for (int e = tid; e < B * B; e += 256) {
                const int p = e / B, q = e % B;
                if (p < bw && q <= p) {
                    double s = 0.0;
                    for (int k = 0; k < n; ++k) {
                        const float* hr = A.H + (size_t)item_at(items, k, A.I) * d + p0;
                        s += (double)hr[p] * (double)hr[q];
                    }
                    Am[e] += s;
                }
            }
            if (tid < bw) {
                double s = 0.0;
                for (int k = 0; k < n; ++k) {
                    const float* hr = A.H + (size_t)item_at(items, k, A.I) * d + p0;
                    s += (yh[k] - (yv ? (double)yv[k] : 1.0)) * (double)hr[tid];
                }
                g[tid] += s;
            }
            __syncthreads();
            for (int k = 0; k < bw; ++k) {
                if (tid == 0) {
                    double v = Am[k * B + k];
                    if (!(v > 0.0)) {
                        *nspd = 1;
                        v = 1.0;
                    }
                    Am[k * B + k] = sqrt(v);
                }
                __syncthreads();
                for (int i = k + 1 + tid; i < bw; i += 256) Am[i * B + k] /= Am[k * B + k];
                __syncthreads();
                const int t = bw - k - 1;
                for (int e = tid; e < t * t; e += 256) {
                    const int i = k + 1 + e / t, j = k + 1 + e % t;
                    if (j <= i) Am[i * B + j] -= Am[i * B + k] * Am[j * B + k];
                }
                __syncthreads();
            }
            if (tid == 0) {
                for (int i = 0; i < bw; ++i) {
                    double s = g[i];
                    for (int k = 0; k < i; ++k) s -= Am[i * B + k] * x[k];
                    x[i] = s / Am[i * B + i];
                }
                for (int i = bw - 1; i >= 0; --i) {
                    double s = x[i];
                    for (int k = i + 1; k < bw; ++k) s -= Am[k * B + i] * x[k];
                    x[i] = s / Am[i * B + i];
                }
            }
            __syncthreads();
            if (tid < bw) w[p0 + tid] -= x[tid];
            for (int k = tid; k < n; k += 256) {
                const float* hr = A.H + (size_t)item_at(items, k, A.I) * d + p0;
                double s = 0.0;
                for (int p = 0; p < bw; ++p) s += x[p] * (double)hr[p];
                yh[k] -= s;
            }
            __syncthreads();
        }
    }
    const float nan = __int_as_float(0x7fc00000);
    for (int f = tid; f < d; f += 256) R.out[f] = *nspd ? nan : (float)w[f];
}

template <int NT, bool GFAC>
__global__ __launch_bounds__(256) void k_foldin(FoldArgs A) {
    constexpr int B = 16 * NT, PB = B + 1, NTL = NT * (NT + 1) / 2;
    extern __shared__ __align__(16) float sm[];
    const int tid = threadIdx.x, lane = tid & 63, q16 = lane & 15, g4 = lane >> 4;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int d = A.d, dp = (d + 3) & ~3;
    float* w = sm;                 // [dp]  the row being folded in
    float* u = w + dp;             // [dp]  alpha0 * w G
    float* part = u + dp;          // [4][B] per-wave gradient partials
    float* dl = part + 4 * B;      // [B]   the step
    int* flag = reinterpret_cast<int*>(dl + B);  // [4]: float64 redo, bad id, not SPD
    float* tail = reinterpret_cast<float*>(flag + 4);  // factors (LDS mode) or the float64 work area

    for (int r = blockIdx.x; r < A.m; r += gridDim.x) {
        const FoldReq R = A.req[r];
        const int n = R.n;
        float* yh = R.ws;
        const int32_t* items = R.copy ? reinterpret_cast<const int32_t*>(R.ws + ws_items_off(n)) : R.items;
        const float* yv = R.y ? (R.copy ? R.ws + ws_y_off(n) : R.y) : nullptr;
        float* fac = GFAC ? R.ws + ws_fac_off(n) : tail;

        // phase 0: w = 0, predictions = 0, inputs staged and checked
        for (int f = tid; f < dp; f += 256) {
            w[f] = 0.f;
            u[f] = 0.f;
        }
        if (tid < 4) flag[tid] = 0;
        __syncthreads();
        for (int k = tid; k < n; k += 256) {
            const int it = R.items[k];
            if ((unsigned)it >= (unsigned)A.I) flag[1] = 1;
            if (R.copy) {
                reinterpret_cast<int32_t*>(R.ws + ws_items_off(n))[k] = it;
                if (R.y) R.ws[ws_y_off(n) + k] = R.y[k];
            }
            yh[k] = 0.f;
        }
        __syncthreads();

        // phase 1: factor every block's Hessian (wave v: blocks v, v+4, ...)
        for (int blk = wave; blk < A.nb; blk += 4) {
            const int p0 = blk * A.b, bw = min(A.b, d - p0);
            floatx4 acc[NTL];
#pragma unroll
            for (int id = 0; id < NTL; ++id) acc[id] = floatx4{0.f, 0.f, 0.f, 0.f};
            for (int k0 = 0; k0 < n; k0 += 4) {
                const int k = k0 + g4;
                const bool v = k < n;
                const float* hr = A.H + (size_t)(v ? item_at(items, k, A.I) : 0) * d + p0;
                float x[NT];
#pragma unroll
                for (int t = 0; t < NT; ++t) {
                    const int c = 16 * t + q16;
                    const float h = hr[c < bw ? c : 0];
                    x[t] = (v && c < bw) ? h : 0.f;
                }
#pragma unroll
                for (int I = 0; I < NT; ++I)
#pragma unroll
                    for (int J = 0; J <= I; ++J) acc[I * (I + 1) / 2 + J] = mfma4(x[I], x[J], acc[I * (I + 1) / 2 + J]);
            }
            float* L = fac + (size_t)blk * B * PB;
            // lower tiles plus alpha0 G[pi,pi] + lambda I (identity on the padding)
#pragma unroll
            for (int I = 0; I < NT; ++I)
#pragma unroll
                for (int J = 0; J <= I; ++J)
#pragma unroll
                    for (int j = 0; j < 4; ++j) {
                        const int row = 16 * I + 4 * g4 + j, col = 16 * J + q16;
                        float v0;
                        if (row < bw && col < bw)
                            v0 = A.alpha0 * A.G[(size_t)(p0 + row) * d + p0 + col] + (row == col ? A.lambda : 0.f);
                        else
                            v0 = (row == col) ? 1.f : 0.f;
                        L[row * PB + col] = acc[I * (I + 1) / 2 + J][j] + v0;
                    }
            wave_fence();
            // Right-looking Cholesky, lane i holding row i: step k scales column k by
            // 1/sqrt(A_kk) and subtracts L_ik L_jk from the later columns j of row i.
            // Entries right of the diagonal are never read (they hold leftovers).
            const int i = lane < B ? lane : 0;
            float a[B];
#pragma unroll
            for (int k = 0; k < B; ++k) a[k] = L[i * PB + k];
            float pmin = 3.0e38f, pmax = 0.f;
#pragma unroll
            for (int k = 0; k < B; ++k) {
                const float piv = readlane(a[k], k);
                if (k < bw) {
                    pmin = fminf(pmin, piv);
                    pmax = fmaxf(pmax, piv);
                }
                const float rs = piv > 0.f ? __builtin_amdgcn_rsqf(piv) : 0.f;
                const float l = a[k] * rs;
                a[k] = l;
#pragma unroll
                for (int j = k + 1; j < B; ++j) a[j] = fmaf(-l, readlane(l, j), a[j]);
            }
            if (lane < B) {
#pragma unroll
                for (int k = 0; k < B; ++k) L[lane * PB + k] = a[k];
            }
            if ((!(pmin > 0.f) || pmin < A.tau * pmax) && lane == 0) flag[0] = 1;
        }
        __syncthreads();

        if (flag[0]) {
            foldin_f64<B>(A, R, n, items, yv, reinterpret_cast<double*>(tail), &flag[2]);
        } else {
            // phase 2: the block steps, sweep after sweep
            const bool vec = (d % 4 == 0) && (A.b % 4 == 0);
            for (int pass = 0; pass < A.passes; ++pass) {
                for (int blk = 0; blk < A.nb; ++blk) {
                    const int p0 = blk * A.b, bw = min(A.b, d - p0);
                    // observed part of the gradient: wave v takes observations v, v+4, ...
                    {
                        const bool cj = lane < bw;
                        float s0 = 0.f, s1 = 0.f;
                        int k = wave;
                        for (; k + 4 < n; k += 8) {
                            const int i0 = item_at(items, k, A.I), i1 = item_at(items, k + 4, A.I);
                            const float r0 = yh[k] - (yv ? yv[k] : 1.f);
                            const float r1 = yh[k + 4] - (yv ? yv[k + 4] : 1.f);
                            const float h0 = A.H[(size_t)i0 * d + p0 + (cj ? lane : 0)];
                            const float h1 = A.H[(size_t)i1 * d + p0 + (cj ? lane : 0)];
                            s0 = fmaf(r0, cj ? h0 : 0.f, s0);
                            s1 = fmaf(r1, cj ? h1 : 0.f, s1);
                        }
                        if (k < n) {
                            const int i0 = item_at(items, k, A.I);
                            const float r0 = yh[k] - (yv ? yv[k] : 1.f);
                            const float h0 = A.H[(size_t)i0 * d + p0 + (cj ? lane : 0)];
                            s0 = fmaf(r0, cj ? h0 : 0.f, s0);
                        }
                        if (lane < B) part[wave * B + lane] = s0 + s1;
                    }
                    __syncthreads();
                    if (wave == 0) {
                        const int i = lane < B ? lane : 0;
                        float g = 0.f;
                        if (lane < bw)
                            g = u[p0 + lane] + A.lambda * w[p0 + lane] +
                                ((part[lane] + part[B + lane]) + (part[2 * B + lane] + part[3 * B + lane]));
                        const float* L = fac + (size_t)blk * B * PB;
                        float lr[B], lc[B];
#pragma unroll
                        for (int k = 0; k < B; ++k) {
                            lr[k] = L[i * PB + k];  // row i of L
                            lc[k] = L[k * PB + i];  // column i of L
                        }
                        const float dinv = 1.f / L[i * PB + i];
                        // L y = g, then L^T delta = y
#pragma unroll
                        for (int k = 0; k < B; ++k) {
                            const float yk = readlane(g, k) * readlane(dinv, k);
                            g = (lane > k) ? fmaf(-lr[k], yk, g) : (lane == k ? yk : g);
                        }
#pragma unroll
                        for (int k = B - 1; k >= 0; --k) {
                            const float xk = readlane(g, k) * readlane(dinv, k);
                            g = (lane < k) ? fmaf(-lc[k], xk, g) : (lane == k ? xk : g);
                        }
                        if (lane < B) dl[lane] = lane < bw ? g : 0.f;
                        if (lane < bw) w[p0 + lane] -= g;
                    }
                    __syncthreads();
                    // u -= alpha0 delta G[pi, :]   and   yhat_k -= <delta, h_k[pi]>
                    for (int f = tid; f < d; f += 256) {
                        float s = 0.f;
                        for (int j = 0; j < bw; ++j) s = fmaf(dl[j], A.G[(size_t)(p0 + j) * d + f], s);
                        u[f] = fmaf(-A.alpha0, s, u[f]);
                    }
                    for (int k = tid; k < n; k += 256) {
                        const float* hr = A.H + (size_t)item_at(items, k, A.I) * d + p0;
                        float s = 0.f;
                        if (vec) {
                            for (int j = 0; j < bw; j += 4) {
                                const float4 h = *reinterpret_cast<const float4*>(hr + j);
                                s = fmaf(dl[j], h.x, s);
                                s = fmaf(dl[j + 1], h.y, s);
                                s = fmaf(dl[j + 2], h.z, s);
                                s = fmaf(dl[j + 3], h.w, s);
                            }
                        } else {
                            for (int j = 0; j < bw; ++j) s = fmaf(dl[j], hr[j], s);
                        }
                        yh[k] -= s;
                    }
                    __syncthreads();
                }
            }
            for (int f = tid; f < d; f += 256) R.out[f] = w[f];
        }
        __syncthreads();
        if (tid == 0) {
            const int st = (flag[0] ? FOLD_ST_FLOAT64 : 0) | (flag[2] ? FOLD_ST_NOT_SPD : 0) |
                           (flag[1] ? FOLD_ST_BAD_ID : 0);
            if (R.st) *R.st = st;
            if (A.cnt) {
                if (flag[1]) atomicAdd(&A.cnt[FOLD_CNT_BAD_ID], 1);
                if (flag[0]) atomicAdd(&A.cnt[FOLD_CNT_FLOAT64], 1);
                if (flag[2]) atomicAdd(&A.cnt[FOLD_CNT_NOT_SPD], 1);
            }
        }
        __syncthreads();
    }
}

constexpr size_t kFoldLdsMax = 150 * 1024;

size_t lds_head_bytes(int32_t d, int32_t B) { return (size_t)(2 * ((d + 3) & ~3) + 5 * B + 4) * 4; }
size_t lds_f64_bytes(int32_t d, int32_t B) { return (size_t)(B * B + ((d + 3) & ~3) + 2 * B) * 8; }
size_t lds_fac_bytes(int32_t nb, int32_t B) { return (size_t)nb * B * (B + 1) * 4; }

template <int NT, bool GFAC>
hipError_t launch_nt(hipStream_t st, const FoldShape& f, const FoldArgs& a) {
    // the dynamic LDS limit is per kernel; set once (thread-safe static initialisation)
    static const hipError_t attr = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_foldin<NT, GFAC>),
                                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)kFoldLdsMax);
    if (attr != hipSuccess) return attr;
    hipLaunchKernelGGL((k_foldin<NT, GFAC>), dim3((unsigned)a.m), dim3(256), f.lds_bytes, st, a);
    return hipGetLastError();
}

}  // namespace

FoldShape fold_shape(int32_t I, int32_t d, int32_t b) {
    FoldShape f;
    f.I = I;
    f.d = d;
    f.b = b;
    f.nb = (d + b - 1) / b;
    f.B = (b + 15) / 16 * 16;
    const size_t head = lds_head_bytes(d, f.B), f64 = lds_f64_bytes(d, f.B), fac = lds_fac_bytes(f.nb, f.B);
    f.gfac = head + std::max(fac, f64) > kFoldLdsMax;
    f.lds_bytes = head + (f.gfac ? f64 : std::max(fac, f64));
    return f;
}

size_t fold_ws_floats(const FoldShape& f, int64_t n) {
    const size_t base = ws_fac_off(n);
    return base + (f.gfac ? ((size_t)f.nb * f.B * (f.B + 1) + 63) / 64 * 64 : 0);
}

hipError_t launch_foldin(hipStream_t st, const FoldShape& f, const float* H, const float* G, float alpha0,
                         float lambda, float tau, int32_t passes, const FoldReq* reqs, int32_t m, int32_t* counters) {
    if (m <= 0) return hipSuccess;
    if (f.lds_bytes > kFoldLdsMax) return hipErrorInvalidValue;
    FoldArgs a{H, G, f.I, f.d, f.b, f.nb, alpha0, lambda, tau, passes, m, reqs, counters};
    switch (f.B) {
        case 16: return f.gfac ? launch_nt<1, true>(st, f, a) : launch_nt<1, false>(st, f, a);
        case 32: return f.gfac ? launch_nt<2, true>(st, f, a) : launch_nt<2, false>(st, f, a);
        case 48: return f.gfac ? launch_nt<3, true>(st, f, a) : launch_nt<3, false>(st, f, a);
        case 64: return f.gfac ? launch_nt<4, true>(st, f, a) : launch_nt<4, false>(st, f, a);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace ials
