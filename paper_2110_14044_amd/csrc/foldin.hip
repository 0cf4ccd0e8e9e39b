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
// request and turned into the block's inverse Hessian (X = L^-1, then X^T X), so
// that a block step is a gradient, one small matrix-vector product and the
// updates, with no sequential solve.
//
// One workgroup (4 wavefronts) per request.  Phase 1: the waves factor and
// invert blocks in parallel (wave v takes blocks v, v+4, ...), keeping X in
// LDS (or in the request's scratch when it does not fit).  Phase 2: the block
// steps in order, one workgroup barrier each: every wave sums its share of the
// gradient, then every wave forms the same step from the four partial sums
// (the same operations in the same order, so the four copies of w agree bit
// for bit).  The ids and residuals yhat - y of a request of up to nl items stay
// in LDS.  A request whose float32 pivots fail the ratio test is redone in
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
    int32_t nl;  // requests of up to nl items keep their ids and residuals in LDS
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
// Factor storage: the packed lower 16 x 16 tiles of a block, rows padded to 17 floats
// so that a lane-per-row and a lane-per-column walk both hit distinct LDS banks.
constexpr int kTP = 17, kTS = 16 * kTP;
__device__ inline int tid_of(int I, int J) { return I * (I + 1) / 2 + J; }
__device__ inline void tile_store(float* T, floatx4 c, int lane) {
#pragma unroll
    for (int j = 0; j < 4; ++j) T[(4 * (lane >> 4) + j) * kTP + (lane & 15)] = c[j];
}
__device__ inline floatx4 tile_load(const float* T, int lane) {
    floatx4 c;
#pragma unroll
    for (int j = 0; j < 4; ++j) c[j] = T[(4 * (lane >> 4) + j) * kTP + (lane & 15)];
    return c;
}
// c += sgn P Q^T and c += sgn P Q for 16 x 16 tiles on the matrix cores
__device__ inline floatx4 mm_pqt(floatx4 c, const float* P, const float* Q, float sgn, int lane) {
#pragma unroll
    for (int s4 = 0; s4 < 4; ++s4) {
        const int o = (lane & 15) * kTP + 4 * s4 + (lane >> 4);
        c = mfma4(sgn * P[o], Q[o], c);
    }
    return c;
}
// c += P^T Q
__device__ inline floatx4 mm_ptq(floatx4 c, const float* P, const float* Q, int lane) {
#pragma unroll
    for (int s4 = 0; s4 < 4; ++s4) {
        const int o = (4 * s4 + (lane >> 4)) * kTP + (lane & 15);
        c = mfma4(P[o], Q[o], c);
    }
    return c;
}
__device__ inline floatx4 mm_pq(floatx4 c, const float* P, const float* Q, float sgn, int lane) {
#pragma unroll
    for (int s4 = 0; s4 < 4; ++s4) {
        const int k = 4 * s4 + (lane >> 4);
        c = mfma4(sgn * P[(lane & 15) * kTP + k], Q[k * kTP + (lane & 15)], c);
    }
    return c;
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
    constexpr int B = 16 * NT, NTL = NT * (NT + 1) / 2;
    extern __shared__ __align__(16) float sm[];
    const int tid = threadIdx.x, lane = tid & 63, q16 = lane & 15, g4 = lane >> 4;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int d = A.d, dp = (d + 3) & ~3, nl = A.nl;
    float* wv = sm;                // [4][dp] each wave's copy of the row being folded in
    float* part = wv + 4 * dp;     // [2][4][B] per-wave gradient partials (double-buffered by step)
    float* gv = part + 8 * B;      // [4][B] per-wave gradient
    float* tv = gv + 4 * B;        // [4][B] per-wave X g
    float* dv = tv + 4 * B;        // [4][B] per-wave step delta
    float* tmp_all = dv + 4 * B;   // [4][kTS] per-wave scratch tile
    int* flag = reinterpret_cast<int*>(tmp_all + 4 * kTS);     // [4]: float64 redo, bad id, not SPD
    int32_t* items_l = reinterpret_cast<int32_t*>(flag + 4);  // [nl] ids of a request of <= nl items
    float* res_l = reinterpret_cast<float*>(items_l + nl);    // [nl] its residuals yhat - y
    float* tail = res_l + nl;      // inverse factors (LDS mode) or the float64 work area
    float* wme = wv + wave * dp;
    float* gme = gv + wave * B;
    float* tme = tv + wave * B;
    float* dme = dv + wave * B;

    for (int r = blockIdx.x; r < A.m; r += gridDim.x) {
        const FoldReq R = A.req[r];
        const int n = R.n;
        const bool in_lds = n <= nl;
        int32_t* ids_w = in_lds ? items_l : reinterpret_cast<int32_t*>(R.ws + ws_items_off(n));
        const int32_t* items = (in_lds || R.copy) ? ids_w : R.items;
        float* res = in_lds ? res_l : R.ws;
        const float* yv = R.y ? (R.copy ? R.ws + ws_y_off(n) : R.y) : nullptr;
        float* fac = GFAC ? R.ws + ws_fac_off(n) : tail;

        // phase 0: w = 0; residuals yhat - y = -y; ids (and labels) staged and checked
        for (int f = tid; f < 4 * dp; f += 256) wv[f] = 0.f;
        if (tid < 4) flag[tid] = 0;
        __syncthreads();
        for (int k = tid; k < n; k += 256) {
            const int it = R.items[k];
            if ((unsigned)it >= (unsigned)A.I) flag[1] = 1;
            const float yk = R.y ? R.y[k] : 1.f;
            if (in_lds || R.copy) ids_w[k] = it;
            if (R.copy && R.y) R.ws[ws_y_off(n) + k] = yk;
            res[k] = -yk;
        }
        __syncthreads();

        // phase 1: every block's Hessian, its Cholesky factor L and X = L^-1
        // (wave v: blocks v, v+4, ...)
        for (int blk = wave; blk < A.nb; blk += 4) {
            const int p0 = blk * A.b, bw = min(A.b, d - p0);
            floatx4 acc[NTL];
#pragma unroll
            for (int id = 0; id < NTL; ++id) acc[id] = floatx4{0.f, 0.f, 0.f, 0.f};
            // 16 MFMA steps of 4 observations per round, their loads issued together
            for (int k0 = 0; k0 < n; k0 += 64) {
                int idr[16];
#pragma unroll
                for (int s16 = 0; s16 < 16; ++s16) {
                    const int k = k0 + 4 * s16 + g4;
                    idr[s16] = k < n ? item_at(items, k, A.I) : -1;
                }
                float x[16][NT];
#pragma unroll
                for (int s16 = 0; s16 < 16; ++s16) {
                    const float* hr = A.H + (size_t)(idr[s16] >= 0 ? idr[s16] : 0) * d + p0;
#pragma unroll
                    for (int t = 0; t < NT; ++t) {
                        const int c = 16 * t + q16;
                        const float h = hr[c < bw ? c : 0];
                        x[s16][t] = (idr[s16] >= 0 && c < bw) ? h : 0.f;
                    }
                }
#pragma unroll
                for (int s16 = 0; s16 < 16; ++s16) {
                    if (k0 + 4 * s16 >= n) break;  // uniform: the rest of the round is empty
#pragma unroll
                    for (int I = 0; I < NT; ++I)
#pragma unroll
                        for (int J = 0; J <= I; ++J)
                            acc[I * (I + 1) / 2 + J] = mfma4(x[s16][I], x[s16][J], acc[I * (I + 1) / 2 + J]);
                }
            }
            float* Lt = fac + (size_t)blk * NTL * kTS;
            // lower tiles plus alpha0 G[pi,pi] + lambda I (identity on the padding); dmax: the
            // largest diagonal entry over the real coordinates (the pivot test's reference)
            float dmax = 0.f;
#pragma unroll
            for (int I = 0; I < NT; ++I)
#pragma unroll
                for (int J = 0; J <= I; ++J) {
                    floatx4 c = acc[I * (I + 1) / 2 + J];
#pragma unroll
                    for (int j = 0; j < 4; ++j) {
                        const int row = 16 * I + 4 * g4 + j, col = 16 * J + q16;
                        if (row < bw && col < bw) {
                            c[j] += A.alpha0 * A.G[(size_t)(p0 + row) * d + p0 + col] + (row == col ? A.lambda : 0.f);
                            if (row == col) dmax = fmaxf(dmax, c[j]);
                        } else {
                            c[j] += (row == col) ? 1.f : 0.f;
                        }
                    }
                    tile_store(Lt + tid_of(I, J) * kTS, c, lane);
                }
            wave_fence();
            // Blocked right-looking Cholesky over the tiles (rolled loops, so the code stays in the
            // instruction cache): the diagonal tile is factored lane-per-row and inverted
            // (Y = L_KK^-1 replaces it), the panel becomes L_IK = A_IK Y^T and the trailing tiles
            // lose L_IK L_JK^T, both on the matrix cores.
            float* tmp = tmp_all + wave * kTS;
            const int i16 = lane & 15;
#pragma unroll
            for (int m = 1; m < 64; m <<= 1) dmax = fmaxf(dmax, __shfl_xor(dmax, m));
            float pmin = 3.0e38f;
            bool nonpos = false;  // a pivot that is not positive, NaN included (fminf skips NaNs)
#pragma unroll 1
            for (int K = 0; K < NT; ++K) {
                float* TK = Lt + tid_of(K, K) * kTS;
                float a[16];
#pragma unroll
                for (int k = 0; k < 16; ++k) a[k] = TK[i16 * kTP + k];
#pragma unroll
                for (int k = 0; k < 16; ++k) {
                    const float piv = readlane(a[k], k);
                    if (16 * K + k < bw) {
                        pmin = fminf(pmin, piv);
                        nonpos = nonpos || !(piv > 0.f);
                    }
                    const float rs = piv > 0.f ? __builtin_amdgcn_rsqf(piv) : 0.f;
                    const float l = a[k] * rs;
                    a[k] = l;
#pragma unroll
                    for (int j = k + 1; j < 16; ++j) a[j] = fmaf(-l, readlane(l, j), a[j]);
                }
                float y[16];
#pragma unroll
                for (int ii = 0; ii < 16; ++ii) {
                    float s0 = 0.f;
#pragma unroll
                    for (int k = 0; k < ii; ++k) s0 = fmaf(readlane(a[k], ii), y[k], s0);
                    const float di = 1.f / readlane(a[ii], ii);
                    y[ii] = (ii < i16) ? 0.f : (ii == i16 ? di : -s0 * di);
                }
                wave_fence();
                if (lane < 16) {
#pragma unroll
                    for (int ii = 0; ii < 16; ++ii) TK[ii * kTP + lane] = y[ii];
                }
                wave_fence();
#pragma unroll 1
                for (int I = K + 1; I < NT; ++I) {
                    float* P = Lt + tid_of(I, K) * kTS;
                    const floatx4 c = mm_pqt(floatx4{0.f, 0.f, 0.f, 0.f}, P, TK, 1.f, lane);
                    wave_fence();
                    tile_store(P, c, lane);
                }
                wave_fence();
#pragma unroll 1
                for (int I = K + 1; I < NT; ++I)
#pragma unroll 1
                    for (int J = K + 1; J <= I; ++J) {
                        float* T = Lt + tid_of(I, J) * kTS;
                        floatx4 c = tile_load(T, lane);
                        c = mm_pqt(c, Lt + tid_of(I, K) * kTS, Lt + tid_of(J, K) * kTS, -1.f, lane);
                        tile_store(T, c, lane);
                    }
                wave_fence();
            }
            // (largest diagonal entry) / (smallest pivot) bounds the block's condition number from
            // below (the pivots lie between the smallest eigenvalue and the diagonal entries)
            if ((nonpos || !(pmin > 0.f) || pmin < A.tau * dmax) && lane == 0) flag[0] = 1;
            // X = L^-1 in place, row by row, each row's tiles in ascending column order:
            // X_II = Y_II (already there) and X_IJ = -Y_II sum_{J <= K < I} L_IK X_KJ.
#pragma unroll 1
            for (int I = 1; I < NT; ++I)
#pragma unroll 1
                for (int J = 0; J < I; ++J) {
                    floatx4 sacc = floatx4{0.f, 0.f, 0.f, 0.f};
#pragma unroll 1
                    for (int K = J; K < I; ++K)
                        sacc = mm_pq(sacc, Lt + tid_of(I, K) * kTS, Lt + tid_of(K, J) * kTS, 1.f, lane);
                    tile_store(tmp, sacc, lane);
                    wave_fence();
                    const floatx4 xv = mm_pq(floatx4{0.f, 0.f, 0.f, 0.f}, Lt + tid_of(I, I) * kTS, tmp, -1.f, lane);
                    wave_fence();
                    tile_store(Lt + tid_of(I, J) * kTS, xv, lane);
                    wave_fence();
                }
            // Hess^-1 = X^T X, lower tiles in place: M_PQ = sum_{I >= P} X_IP^T X_IQ.  Going
            // through P, then Q, ascending, no X tile is overwritten before its last use.
#pragma unroll 1
            for (int P = 0; P < NT; ++P)
#pragma unroll 1
                for (int Q = 0; Q <= P; ++Q) {
                    floatx4 macc = floatx4{0.f, 0.f, 0.f, 0.f};
#pragma unroll 1
                    for (int I = P; I < NT; ++I)
                        macc = mm_ptq(macc, Lt + tid_of(I, P) * kTS, Lt + tid_of(I, Q) * kTS, lane);
                    wave_fence();
                    tile_store(Lt + tid_of(P, Q) * kTS, macc, lane);
                    wave_fence();
                }
        }
        __syncthreads();

        if (flag[0]) {
            foldin_f64<B>(A, R, n, items, yv, reinterpret_cast<double*>(tail), &flag[2]);
        } else {
            // phase 2: the block steps, sweep after sweep.  Each wave sums its part of the
            // gradient (a quarter of the rows of G, every fourth observation), then every wave
            // forms the same step from the four partials and applies it to its own copy of w,
            // so one barrier per step suffices.  A wave also owns the residuals of its
            // observations: it applies the previous step to them just before they are used.
            const bool vec = (d % 4 == 0) && (A.b % 4 == 0);
            const int nv = n > wave ? (n - wave + 3) / 4 : 0;  // observations wave, wave+4, ...
            const int fq = (d + 3) / 4, f_lo = min(d, wave * fq), f_hi = min(d, f_lo + fq);
            int step = 0, pp0 = 0, pbw = 0;
            for (int pass = 0; pass < A.passes; ++pass) {
                for (int blk = 0; blk < A.nb; ++blk, ++step) {
                    const int p0 = blk * A.b, bw = min(A.b, d - p0);
                    const float* Xt = fac + (size_t)blk * NTL * kTS;
                    const int col = p0 + (lane < bw ? lane : 0);
                    // dense part: alpha0 sum_f w_f G[f][p0 + lane] over this wave's rows f
                    float sd0 = 0.f, sd1 = 0.f;
                    for (int f = f_lo; f < f_hi; f += 64) {
                        float gg[64];
#pragma unroll
                        for (int q = 0; q < 64; ++q) gg[q] = A.G[(size_t)min(f + q, f_hi - 1) * d + col];
#pragma unroll
                        for (int q = 0; q < 64; q += 2) {
                            const float w0 = (f + q < f_hi) ? wme[f + q] : 0.f;
                            const float w1 = (f + q + 1 < f_hi) ? wme[f + q + 1] : 0.f;
                            sd0 = fmaf(w0, gg[q], sd0);
                            sd1 = fmaf(w1, gg[q + 1], sd1);
                        }
                    }
                    // observations: previous step applied to the residuals, then res_k h_k[p0 + lane].
                    // Every load of a round (the previous block's row for the residual update, the
                    // current block's values for the gradient) is issued before any is used.
                    float so0 = 0.f, so1 = 0.f;
                    for (int m0 = 0; m0 < nv; m0 += 64) {
                        const int k = wave + 4 * (m0 + lane);
                        const bool kv = k < n;
                        const int itl = kv ? item_at(items, k, A.I) : 0;
                        float rl = kv ? res[k] : 0.f;
                        const int cnt = min(64, nv - m0);
                        float hg[64];
#pragma unroll
                        for (int s8 = 0; s8 < 64; ++s8) {
                            const int it = __builtin_amdgcn_readlane(itl, s8);
                            hg[s8] = (s8 < cnt) ? A.H[(size_t)it * d + col] : 0.f;
                        }
                        if (step > 0) {
                            const float* hr = A.H + (size_t)itl * d + pp0;
                            float e0 = 0.f, e1 = 0.f;
                            if (vec) {
                                float4 hv[16];
#pragma unroll
                                for (int j4 = 0; j4 < 16; ++j4)
                                    hv[j4] = (4 * j4 < pbw) ? *reinterpret_cast<const float4*>(hr + 4 * j4)
                                                            : float4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
                                for (int j4 = 0; j4 < 16; ++j4) {
                                    const float4 dd = *reinterpret_cast<const float4*>(dme + 4 * j4);
                                    e0 = fmaf(dd.x, hv[j4].x, e0);
                                    e1 = fmaf(dd.y, hv[j4].y, e1);
                                    e0 = fmaf(dd.z, hv[j4].z, e0);
                                    e1 = fmaf(dd.w, hv[j4].w, e1);
                                }
                            } else {
                                for (int j = 0; j < pbw; ++j) e0 = fmaf(dme[j], hr[j], e0);
                            }
                            rl -= e0 + e1;
                            if (kv) res[k] = rl;
                        }
#pragma unroll
                        for (int s8 = 0; s8 < 64; s8 += 2) {
                            so0 = fmaf(readlane(rl, s8), hg[s8], so0);
                            so1 = fmaf(readlane(rl, s8 + 1), hg[s8 + 1], so1);
                        }
                    }
                    float* pb = part + (step & 1) * 4 * B;
                    if (lane < B) pb[wave * B + lane] = lane < bw ? A.alpha0 * (sd0 + sd1) + (so0 + so1) : 0.f;
                    __syncthreads();
                    // every wave: gradient, delta = X^T (X g) = Hess^-1 g, its copy of w updated
                    if (lane < B)
                        gme[lane] = lane < bw ? ((pb[lane] + pb[B + lane]) + (pb[2 * B + lane] + pb[3 * B + lane])) +
                                                    A.lambda * wme[p0 + lane]
                                              : 0.f;
                    wave_fence();
                    (void)tme;
                    // delta = Hess^-1 g with the inverse's lower tiles: lane p walks row p of the tiles
                    // left of (and on) the diagonal and column p of the tiles below it
                    const int i = lane < B ? lane : 0;
                    const int Ii = i >> 4, ri = i & 15;
                    float t4[4] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
                    for (int K = 0; K < NT; ++K) {
                        const bool below = K > Ii;
                        const float* tp = Xt + (below ? tid_of(K, Ii) : tid_of(Ii, K)) * kTS;
#pragma unroll
                        for (int kk = 0; kk < 16; ++kk) {
                            const float v = below ? tp[kk * kTP + ri] : tp[ri * kTP + kk];
                            t4[kk & 3] = fmaf(v, gme[16 * K + kk], t4[kk & 3]);
                        }
                    }
                    const float del = (t4[0] + t4[1]) + (t4[2] + t4[3]);
                    if (lane < B) dme[lane] = lane < bw ? del : 0.f;
                    if (lane < bw) wme[p0 + lane] -= del;
                    wave_fence();
                    pp0 = p0;
                    pbw = bw;
                }
            }
            if (wave == 0)
                for (int f = lane; f < d; f += 64) R.out[f] = wme[f];
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

size_t lds_head_bytes(int32_t d, int32_t B, int32_t nl) {
    return (size_t)(4 * ((d + 3) & ~3) + 20 * B + 4 * kTS + 4 + 2 * nl) * 4;
}
size_t lds_f64_bytes(int32_t d, int32_t B) { return (size_t)(B * B + ((d + 3) & ~3) + 2 * B) * 8; }
size_t lds_fac_bytes(int32_t nb, int32_t B) {
    const int nt = B / 16;
    return (size_t)nb * (nt * (nt + 1) / 2) * kTS * 4;
}

template <int NT, bool GFAC>
hipError_t launch_nt(hipStream_t st, const FoldShape& f, const FoldArgs& a) {
    // raises the kernel's dynamic-LDS limit on this device the first time (the limit is per device)
    static OccCache occ;
    (void)resident_per_cu(occ, reinterpret_cast<const void*>(&k_foldin<NT, GFAC>), 256, kFoldLdsMax, true, 1);
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
    const size_t f64 = lds_f64_bytes(d, f.B), fac = lds_fac_bytes(f.nb, f.B);
    static const int32_t kNl[] = {2048, 1024, 256, 0};
    for (int gfac = 0; gfac < 2; ++gfac) {
        const size_t rest = gfac ? f64 : std::max(fac, f64);
        for (int32_t nl : kNl) {
            const size_t bytes = lds_head_bytes(d, f.B, nl) + rest;
            if (bytes <= kFoldLdsMax) {
                f.gfac = gfac != 0;
                f.nl = nl;
                f.lds_bytes = bytes;
                return f;
            }
        }
    }
    f.gfac = true;
    f.nl = 0;
    f.lds_bytes = lds_head_bytes(d, f.B, 0) + f64;  // above the limit: launch_foldin refuses it
    return f;
}

size_t fold_ws_floats(const FoldShape& f, int64_t n) {
    const size_t base = ws_fac_off(n);
    return base + (f.gfac ? (lds_fac_bytes(f.nb, f.B) / 4 + 63) / 64 * 64 : 0);
}

hipError_t launch_foldin(hipStream_t st, const FoldShape& f, const float* H, const float* G, float alpha0,
                         float lambda, float tau, int32_t passes, const FoldReq* reqs, int32_t m, int32_t* counters) {
    if (m <= 0) return hipSuccess;
    if (f.lds_bytes > kFoldLdsMax) return hipErrorInvalidValue;
    FoldArgs a{H, G, f.I, f.d, f.b, f.nb, alpha0, lambda, tau, passes, m, f.nl, reqs, counters};
    switch (f.B) {
        case 16: return f.gfac ? launch_nt<1, true>(st, f, a) : launch_nt<1, false>(st, f, a);
        case 32: return f.gfac ? launch_nt<2, true>(st, f, a) : launch_nt<2, false>(st, f, a);
        case 48: return f.gfac ? launch_nt<3, true>(st, f, a) : launch_nt<3, false>(st, f, a);
        case 64: return f.gfac ? launch_nt<4, true>(st, f, a) : launch_nt<4, false>(st, f, a);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace ials
