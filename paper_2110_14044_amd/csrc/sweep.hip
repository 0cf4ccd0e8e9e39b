// The block pass of iALS++ (sec. 4, eq. 8-9, Alg. 3) on gfx950.
//
// For every row r of the side being updated (users, or items) and the block
// pi = [p0, p0+bw) padded to B = 16*NT columns:
//   T      = X_other[partners(r), pi]            gathered straight from the embedding table
//   yhat_k = c_k + <x_{r,pi}, T_k>               (c: prediction cache without block pi)
//   Hess   = alpha0 G_pipi + lambda I + T^T diag(a) T   (MFMA f32 16x16x4, lower tiles only)
//   grad   = R0[r] + T^T (a (yhat - y))          (R0 = alpha0 x_r G^pi + lambda x_{r,pi}, precomputed)
//   delta  = Hess^-1 grad                         (blocked LDL^T on the accumulator tiles)
//   x_{r,pi} -= delta
//
// The prediction cache holds, per observation, the prediction minus the part of
// the current block (c = yhat - <x_pi, o_pi>).  It does not change while block
// pi is being optimised, so no pass has to patch it: each pass forms yhat from
// c and the two rows it already holds.  The first pass of a new block pi' moves
// the cache: yhat = c + <x_pi, o_pi> (the old block, one more gather) and
// c' = yhat - <x_pi', o_pi'>.  This is the same iteration as the delta update of
// the cached predictions in Alg. 3 (the predictions are equal in exact arithmetic).
//
// Rows longer than the segment length are split into segments: k_sweep_seg
// accumulates each segment's partial Hessian and gradient, the row kernel adds
// them in segment order (a fixed order, so results are bitwise reproducible) and
// solves.
// A row whose float32 pivots (the diagonal of D in Hess = L D L^T, the squares of the
// Cholesky diagonal) fall below tau * (largest pivot), or are
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
#include <atomic>
#include <cmath>

#include "ials_internal.h"

namespace ials {
namespace {



__device__ inline floatx4 mfma4(float a, float b, floatx4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
// bfloat16 (round to nearest even) of four floats, packed as the 4-element operand of
// v_mfma_f32_16x16x16_bf16 (element v stands for observation v of this lane's four); the
// conversions are the hardware's v_cvt_pk_bf16_f32, two floats per instruction.
__device__ inline shortx4 bf16x4(float a, float b, float c, float d) {
    typedef __bf16 bf16x4_t __attribute__((ext_vector_type(4)));
    const bf16x4_t v = {(__bf16)a, (__bf16)b, (__bf16)c, (__bf16)d};
    return __builtin_bit_cast(shortx4, v);
}
__device__ inline floatx4 mfma_bf16(shortx4 a, shortx4 b, floatx4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
}
__device__ inline float readlane(float x, int l) {
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x), l));
}
// Order LDS accesses of one wavefront (LDS operations of a wave execute in order).
__device__ inline void wave_lds_fence() {
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
}
// Next item from a work queue shared by all wavefronts.  The first active lane
// takes the item and broadcasts it, so the protocol holds for any exec mask.
__device__ inline int queue_next(int32_t* cursor, int lane) {
    const unsigned long long active = __ballot(1);
    const int leader = __ffsll((long long)active) - 1;
    int it = 0;
    if (lane == leader) it = atomicAdd(cursor, 1);
    return __builtin_amdgcn_readfirstlane(it);
}
__device__ inline float sum16(float s) { return row_sum16(s); }

template <int NT>
constexpr int ntiles() { return NT * (NT + 1) / 2; }

// floats of one segment partial: NTL tiles x 64 lanes x 4 + B gradient entries
template <int NT>
constexpr int seg_stride() { return ntiles<NT>() * 256 + 16 * NT; }

template <int NT, bool FULL>
__host__ __device__ constexpr int colmap(int p) { return FULL ? NT * (p & 15) + (p >> 4) : p; }

// x[t] = X[i][p0 + column of position 16 t + q16], 0 outside the block [p0, p0+bw).
// Vector mode: lane q16 takes the NT consecutive columns NT*q16 .. NT*q16+NT-1.
template <int NT, bool VEC>
__device__ inline void load_cols(const float* __restrict__ X, int d, int i, int p0, int bw, int q16, float* x) {
    const float* xr = X + (size_t)i * d + p0;
    if constexpr (VEC && NT == 8) {
        const float4 v0 = *reinterpret_cast<const float4*>(xr + 8 * q16);
        const float4 v1 = *reinterpret_cast<const float4*>(xr + 8 * q16 + 4);
        x[0] = v0.x;
        x[1] = v0.y;
        x[2] = v0.z;
        x[3] = v0.w;
        x[4] = v1.x;
        x[5] = v1.y;
        x[6] = v1.z;
        x[7] = v1.w;
    } else if constexpr (VEC && NT == 4) {
        const float4 v = *reinterpret_cast<const float4*>(xr + 4 * q16);
        x[0] = v.x;
        x[1] = v.y;
        x[2] = v.z;
        x[3] = v.w;
    } else if constexpr (VEC && NT == 2) {
        const float2 v = *reinterpret_cast<const float2*>(xr + 2 * q16);
        x[0] = v.x;
        x[1] = v.y;
    } else if constexpr (VEC && NT == 1) {
        x[0] = xr[q16];
    } else {
#pragma unroll
        for (int t = 0; t < NT; ++t) {
            const int c = 16 * t + q16;
            const float v = xr[c < bw ? c : bw - 1];
            x[t] = (c < bw) ? v : 0.f;
        }
    }
}

// The current block of the cache, read in vector mode when it is a full block.
template <int NT>
__device__ inline void load_cur(const SweepArgs& A, const float* X, int i, int q16, float* x) {
    if (A.cur_full)
        load_cols<NT, (NT != 3)>(X, A.d, i, A.pc, A.bwc, q16, x);
    else
        load_cols<NT, false>(X, A.d, i, A.pc, A.bwc, q16, x);
}

// acc (lower tiles, MFMA D layout, p order) += T^T diag(a) T and gp[t] (position
// 16t+q16, this lane group's share) += T^T (a (yhat - y)) over observations
// [lo, hi) of one row whose own block values are own[] (block pi) and ownc[]
// (the cache's block, TRANS only).  With TRANS the cache entries are moved to pi.
// BF: the Hessian products take bfloat16 operands (one 16x16x16 MFMA per tile for the
// four observations of every lane group, 16 in all); the gradient and the predictions
// stay float32.
// CF: the cache's block is a full block (vector loads of the partner rows' old block, no
// per-step branch between the two load forms).
template <int NT, bool FULL, bool TRANS, bool BF, int U = 4, bool CF = true>
__device__ inline void accumulate(const SweepArgs& A, int64_t lo, int64_t hi, const float* own, const float* ownc,
                                  floatx4* acc, float* gp, int lane) {
    // U steps of 4 observations per batch.  A batch has no branches: its partner rows are
    // all loaded before any is used (steps past the chunk load a valid row and contribute
    // nothing, their weight being 0), so the loads of a batch are in flight together.
    static_assert(U == 2 || U == 4 || U == 8, "batches of 2, 4 or 8 steps");
    // a bfloat16 product takes four steps (K = 16: four values per lane group); with two-step
    // batches the product's other two values are zero (half the product unused, for registers)
    constexpr int BFS = U < 4 ? 2 : 4;
    static_assert(!BF || U % BFS == 0, "bfloat16 products of two or four steps");
    const int q16 = lane & 15, g4 = lane >> 4;
    for (int64_t c0 = lo; c0 < hi; c0 += 64) {
        const int64_t k = c0 + lane;
        const bool v = k < hi;
        // Per observation (one per lane): the partner id, the cache slot, the cache entry less
        // the label (with TRANS the cache entry and the label apart) and the weight, 0 past
        // the chunk, so that padding steps add nothing without a test of their own.
        int ci = 0, si = 0;
        float cv = 0.f, yv = 1.f, av = TRANS ? 1.f : 0.f;
        if (v) {
            ci = A.col[k];
            si = A.slot ? A.slot[k] : (int)k;
            cv = A.cache[si];
            if (A.y) yv = A.y[k];
            if constexpr (TRANS) {
                if (A.a) av = A.a[k];
            } else {
                av = A.a ? A.a[k] : 1.f;
            }
        }
        if constexpr (!TRANS) cv -= yv;
        const int cnt = (int)std::min<int64_t>(64, hi - c0);
        const int nsteps = (cnt + 3) >> 2;
        for (int st = 0; st < nsteps; st += U) {
            float x[U][NT], xc[U][TRANS ? NT : 1];
            float xa4[BF ? U : 1][NT];
            // Without TRANS: ds_bpermute byte address of lane 4 st + g4, the observation of
            // step st in this lane group (step st + u at +16 u; st + u < 16, so no wrap), and
            // the label and the padding folded into the permuted values.  The passes that move
            // the cache keep lane-index shuffles, the label and weight permuted only when
            // given and the validity test their cache store needs anyway (the same form with
            // the folded values measured slower there).
            const int sa = 16 * st + 4 * g4;
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int i = TRANS ? __shfl(ci, (4 * (st + u) + g4) & 63) : __builtin_amdgcn_ds_bpermute(sa + 16 * u, ci);
                load_cols<NT, FULL>(A.Xo, A.d, i, A.p0, A.bw, q16, x[u]);
                if constexpr (TRANS) {
                    if constexpr (CF)
                        load_cols<NT, (NT != 3)>(A.Xo, A.d, i, A.pc, A.bwc, q16, xc[u]);
                    else
                        load_cols<NT, false>(A.Xo, A.d, i, A.pc, A.bwc, q16, xc[u]);
                }
            }
#pragma unroll
            for (int u = 0; u < U; ++u) {
                // residual yhat - y: with TRANS from the cache's block, else from this block
                float ak, res, sp = 0.f;
                if constexpr (TRANS) {
                    const int src = 4 * (st + u) + g4;
                    const bool valid = src < cnt;
                    const float ck = __shfl(cv, src & 63);
                    const float yk = A.y ? __shfl(yv, src & 63) : 1.f;
                    const float ak_all = A.a ? __shfl(av, src & 63) : 1.f;
                    ak = valid ? ak_all : 0.f;
#pragma unroll
                    for (int t = 0; t < NT; ++t) sp = fmaf(x[u][t], own[t], sp);
                    sp = sum16(sp);
                    float sc = 0.f;
#pragma unroll
                    for (int t = 0; t < NT; ++t) sc = fmaf(xc[u][t], ownc[t], sc);
                    sc = sum16(sc);
                    const float yh = ck + sc;
                    res = yh - yk;
                    const int sk = __shfl(si, src & 63);
                    if (q16 == 0 && valid) A.cache[sk] = yh - sp;
                } else {
                    const int sau = sa + 16 * u;
                    const float ck = __int_as_float(__builtin_amdgcn_ds_bpermute(sau, __float_as_int(cv)));
                    ak = __int_as_float(__builtin_amdgcn_ds_bpermute(sau, __float_as_int(av)));
#pragma unroll
                    for (int t = 0; t < NT; ++t) sp = fmaf(x[u][t], own[t], sp);
                    sp = sum16(sp);
                    res = ck + sp;
                }
                const float rk = ak * res;
                float xa[NT];
#pragma unroll
                for (int t = 0; t < NT; ++t) {
                    gp[t] = fmaf(rk, x[u][t], gp[t]);
                    xa[t] = ak * x[u][t];
                }
                if constexpr (BF) {
#pragma unroll
                    for (int t = 0; t < NT; ++t) xa4[u][t] = xa[t];
                } else {
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
            if constexpr (BF) {
                // four steps per bfloat16 product; a weight of 0 zeroes a padding step's terms
#pragma unroll
                for (int h = 0; h < U; h += BFS) {
                    shortx4 pa[NT], pb[NT];
#pragma unroll
                    for (int t = 0; t < NT; ++t) {
                        if constexpr (BFS == 4) {
                            pa[t] = bf16x4(xa4[h][t], xa4[h + 1][t], xa4[h + 2][t], xa4[h + 3][t]);
                            pb[t] = bf16x4(x[h][t], x[h + 1][t], x[h + 2][t], x[h + 3][t]);
                        } else {
                            pa[t] = bf16x4(xa4[h][t], xa4[h + 1][t], 0.f, 0.f);
                            pb[t] = bf16x4(x[h][t], x[h + 1][t], 0.f, 0.f);
                        }
                    }
                    int id = 0;
#pragma unroll
                    for (int ti = 0; ti < NT; ++ti)
#pragma unroll
                        for (int tj = 0; tj <= ti; ++tj) {
                            acc[id] = mfma_bf16(pa[ti], pb[tj], acc[id]);
                            ++id;
                        }
                }
            }
        }
    }
}

// Steps per batch of partner-row loads (4 rows a step): 4, or 2 when the pass also loads the
// cache's block of every partner row in float32 (the registers of 4 would spill).
template <bool TRANS, bool BF>
constexpr int kBatchSteps = (TRANS && !BF) ? 2 : 4;

// Own block values of row r: own[t] at block pi (this pass's column order),
// ownc[t] at the cache's block (TRANS only).
template <int NT, bool FULL, bool TRANS>
__device__ inline void load_own(const SweepArgs& A, int r, int q16, float* own, float* ownc) {
    load_cols<NT, FULL>(A.X, A.d, r, A.p0, A.bw, q16, own);
    if constexpr (TRANS) load_cur<NT>(A, A.X, r, q16, ownc);
}

template <int NT, bool FULL, bool TRANS, bool BF, bool CF>
__global__ __launch_bounds__(256) void k_sweep_seg(SweepArgs A) {
    constexpr int NTL = ntiles<NT>();
    const int lane = threadIdx.x & 63, q16 = lane & 15, g4 = lane >> 4;
    // the wavefront index made uniform, so that the segment and row indices, the row bounds and
    // the loops over them live in scalar registers
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    for (int j = blockIdx.x * 4 + wave; j < A.nseg; j += gridDim.x * 4) {
        const int it = A.seg_order[j];
        floatx4 acc[NTL];
        float gp[NT], own[NT], ownc[TRANS ? NT : 1];
#pragma unroll
        for (int id = 0; id < NTL; ++id) acc[id] = floatx4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int t = 0; t < NT; ++t) gp[t] = 0.f;
        load_own<NT, FULL, TRANS>(A, A.seg_row[it], q16, own, ownc);
        accumulate<NT, FULL, TRANS, BF, kBatchSteps<TRANS, BF>, CF>(A, A.seg_lo[it], A.seg_hi[it], own, ownc, acc, gp, lane);
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

// Group sums of segment partials.  A row of ns segments has ceil(ns / G) groups of G
// consecutive segments (G = A.seg_group); the partial of each group's first segment becomes
// the sum of the group's partials, element by element in segment order, so the row kernel
// adds ceil(ns / G) partials instead of ns (one wavefront would otherwise sum a very long
// row's partials alone).  Block (s, y) covers 1,024 floats of segment s's partial.
__global__ __launch_bounds__(256) void k_seg_group(SweepArgs A, int32_t stride) {
    const int s = blockIdx.x;
    const int r = A.seg_row[s];
    const int sf = A.seg_first[r];
    if ((s - sf) % A.seg_group != 0) return;
    const int64_t len = A.ptr[r + 1] - A.ptr[r];
    const int ns = (int)((len + A.seg_len - 1) / A.seg_len);
    const int end = std::min(s + A.seg_group, sf + ns);
    const int e = (blockIdx.y * 256 + threadIdx.x) * 4;
    if (end - s < 2 || e >= stride) return;
    float* P = A.seg_part + (size_t)s * stride + e;
    float4 v = *reinterpret_cast<const float4*>(P);
    int t = s + 1;
    // four partials loaded together, then added in segment order
    for (; t + 4 <= end; t += 4) {
        float4 w[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) w[j] = *reinterpret_cast<const float4*>(A.seg_part + (size_t)(t + j) * stride + e);
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            v.x += w[j].x;
            v.y += w[j].y;
            v.z += w[j].z;
            v.w += w[j].w;
        }
    }
    for (; t < end; ++t) {
        const float4 w = *reinterpret_cast<const float4*>(A.seg_part + (size_t)t * stride + e);
        v.x += w.x;
        v.y += w.y;
        v.z += w.z;
        v.w += w.w;
    }
    *reinterpret_cast<float4*>(P) = v;
}

// Blocked factorisation storage: panel K (16 columns, rows 16K..B-1) of the factor L is
// kept in LDS, panels packed one after another.  The 128-wide kernel keeps one panel at a
// row stride of kPS = 20 floats, which keeps rows 16-byte aligned and spreads the accesses
// over the banks (the accumulator-layout stores, rows 4 apart in a half-wave; the
// lane-per-row 16-byte loads; the operand loads of the trailing updates).  The narrow kernel
// keeps all of its panels for the back substitution at a stride of kPN = 16 floats: 10 KB
// per wavefront, so that four 4-wavefront blocks fit a CU's 160 KB of LDS and each SIMD
// holds four wavefronts (with a stride of 20 it held three; the accumulator-layout stores
// and the trailing-update operand loads then meet 4-way bank conflicts, which cost less
// than the fourth wavefront gains).
constexpr int kPS = 20;
constexpr int kPN = 16;
template <int NT>
constexpr int panel_rows() { return 16 * NT * (NT + 1) / 2; }
template <int NT>
__host__ __device__ constexpr int panel_row0(int K) { return 16 * (K * NT - K * (K - 1) / 2); }
template <int NT>
constexpr int rows_lds_floats_per_wave() { return panel_rows<NT>() * kPN; }
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

// Steps KK..15 of panel K (see ldl_solve).  src: ds_bpermute address of the lane of row
// group K in this lane's row position; lk = this lane's row - 16K (-1 - 16K past the block).
// piv and D were read for this step by the previous one: each step updates column k + 1
// first and at once reads the next pivot and starts the next copy of the pivot column, so
// that their latency runs under the step's other column updates (look-ahead).
template <int K, int KK>
__device__ inline void panel_steps(float* p, float& g, float& mypiv, float lk, int src, float piv, float D) {
    if constexpr (KK < 16) {
        constexpr int k = 16 * K + KK;
        // lane k keeps the pivot
        asm volatile("s_nop 1\n\tv_writelane_b32 %0, %1, %2" : "+v"(mypiv) : "s"(piv), "i"(k));
        const float nr = __builtin_amdgcn_rcpf(-piv);
        const float act = __builtin_amdgcn_fmed3f(lk - (float)KK, 0.f, 1.f);  // 1 in the lanes below row k
        const float tn = p[KK] * nr * act;              // -t_i
        float pivn = 0.f, Dn = 0.f;
        if constexpr (KK < 15) {
            fmac_rowbcast<KK + 1, true>(p[KK + 1], D, tn);
            pivn = readlane(p[KK + 1], k + 1);
            if constexpr (KK < 14) Dn = __int_as_float(__builtin_amdgcn_ds_bpermute(src, __float_as_int(p[KK + 1])));
            // keep the reads of the next step ahead of this step's other updates
            __builtin_amdgcn_sched_barrier(0);
            eliminate_cols<KK + 2, false>(p, D, tn);
        }
        g = fmaf(tn, readlane(g, k), g);
        p[KK] = tn;
        panel_steps<K, KK + 1>(p, g, mypiv, lk, src, pivn, Dn);
    }
}

// Solve Hess x = g for one row with the Hessian in the accumulator tiles (lower tiles, p
// order) and lane p < B holding g_p: a blocked right-looking LDL^T factorisation with the
// forward substitution folded in, then the back substitution.  Returns false (in every lane)
// when a pivot is not positive or below tau * (largest pivot) over the real coordinates.
//
// Panel K (16 columns) is moved to the lane-per-row layout through LDS (lane i holds
// A_{i, 16K..16K+15} in p[]).  Step k = 16K + kk: piv = A_kk; lanes i > k take
// t_i = A_ik / piv (0 in the other lanes), g_i -= t_i g_k and A_ij -= t_i A_jk for the
// panel's later columns j, where column k of the diagonal tile (held by the lanes of row
// group K) is first copied to every row group and then read with a row broadcast.  Lane i
// keeps -t_i in place of A_ik, so a finished panel holds -L (unit lower factor, zeros on and
// above the diagonal), which the back substitution reads column-wise.  The trailing tiles
// take A_IJ -= L_IK diag(piv) L_JK^T on the matrix cores.
template <int NT, int K>
__device__ inline void ldl_panels(floatx4* acc, float& g, float* pan, int ln, float li, float& mypiv) {
    if constexpr (K < NT) {
        constexpr int B = 16 * NT;
        const int lane = threadIdx.x & 63, q16 = lane & 15, g4 = lane >> 4;
        float* PK = pan + panel_row0<NT>(K) * kPN;  // row r >= 16K at PK + (r - 16K) * kPN
#pragma unroll
        for (int I = K; I < NT; ++I) {
            const int id = I * (I + 1) / 2 + K;
#pragma unroll
            for (int j = 0; j < 4; ++j) PK[(16 * (I - K) + 4 * g4 + j) * kPN + q16] = acc[id][j];
        }
        wave_lds_fence();
        const bool mine = (ln >= 16 * K) && (ln < B);
        const int prow = mine ? ln - 16 * K : 0;
        float p[16];
#pragma unroll
        for (int c4 = 0; c4 < 4; ++c4) {
            const float4 v = *reinterpret_cast<const float4*>(PK + prow * kPN + 4 * c4);
            p[4 * c4 + 0] = v.x;
            p[4 * c4 + 1] = v.y;
            p[4 * c4 + 2] = v.z;
            p[4 * c4 + 3] = v.w;
        }
        wave_lds_fence();
        {
            const int src = (16 * K + (ln & 15)) * 4;
            const float piv0 = readlane(p[0], 16 * K);
            const float D0 = __int_as_float(__builtin_amdgcn_ds_bpermute(src, __float_as_int(p[0])));
            panel_steps<K, 0>(p, g, mypiv, li - 16.f * K, src, piv0, D0);
        }
        if (mine) {
#pragma unroll
            for (int c4 = 0; c4 < 4; ++c4)
                *reinterpret_cast<float4*>(PK + prow * kPN + 4 * c4) =
                    make_float4(p[4 * c4], p[4 * c4 + 1], p[4 * c4 + 2], p[4 * c4 + 3]);
        }
        wave_lds_fence();
        // trailing tiles: A_IJ -= L_IK diag(piv) L_JK^T for K < J <= I (the panel holds -L)
        if constexpr (K + 1 < NT) {
#pragma unroll
            for (int s4 = 0; s4 < 4; ++s4) {
                const float npm = -__int_as_float(
                    __builtin_amdgcn_ds_bpermute((16 * K + 4 * s4 + g4) * 4, __float_as_int(mypiv)));
                float op[NT];
#pragma unroll
                for (int I = K + 1; I < NT; ++I) op[I] = PK[(16 * (I - K) + q16) * kPN + 4 * s4 + g4];
#pragma unroll
                for (int I = K + 1; I < NT; ++I) {
                    const float a = op[I] * npm;
#pragma unroll
                    for (int J = K + 1; J <= I; ++J) {
                        const int id = I * (I + 1) / 2 + J;
                        acc[id] = mfma4(a, op[J], acc[id]);
                    }
                }
            }
        }
        __builtin_amdgcn_sched_barrier(0);
        ldl_panels<NT, K + 1>(acc, g, pan, ln, li, mypiv);
    }
}

// Largest diagonal entry of the Hessian over the real coordinates (lower tiles in p order,
// the accumulator layout: lane (q16, g4) holds row 4 g4 + j, column q16 of each tile, so its
// diagonal element of a diagonal tile, if any, is register q16 - 4 g4).  Every lane gets it.
template <int NT, bool FULL>
__device__ inline float diag_max(const floatx4* acc, int lane, int bw) {
    const int q16 = lane & 15, jd = q16 - 4 * (lane >> 4);
    float dmax = 0.f;
#pragma unroll
    for (int t = 0; t < NT; ++t) {
        const floatx4 v = acc[t * (t + 3) / 2];
        const float e = jd == 0 ? v[0] : (jd == 1 ? v[1] : (jd == 2 ? v[2] : v[3]));
        if (jd >= 0 && jd < 4 && colmap<NT, FULL>(16 * t + q16) < bw) dmax = fmaxf(dmax, e);
    }
#pragma unroll
    for (int m = 1; m < 64; m <<= 1) dmax = fmaxf(dmax, __shfl_xor(dmax, m));
    return dmax;
}

template <int NT, bool FULL>
__device__ inline bool ldl_solve(floatx4* acc, float g, float* pan, int ln, float tau,
                                 int my_col, int bw, float& x) {
    constexpr int B = 16 * NT;
    const float li = (ln < B) ? (float)ln : -1.f;  // lanes past the block never take a step
    float mypiv = 1.f;                             // lane k: the pivot of step k
    // the pivots D_k of Hess = L D L^T lie between the smallest eigenvalue and the diagonal
    // entries, so (largest diagonal entry) / (smallest pivot) bounds the condition number
    // from below; a row is redone in float64 when it exceeds 1 / tau
    const float dmax = diag_max<NT, FULL>(acc, ln, bw);
    ldl_panels<NT, 0>(acc, g, pan, ln, li, mypiv);
    // pivot check over the real (unpadded) coordinates
    const bool real = (ln < B) && (my_col < bw);
    float pmin = real ? mypiv : 3.0e38f;
#pragma unroll
    for (int m = 1; m < 64; m <<= 1) pmin = fminf(pmin, __shfl_xor(pmin, m));
    // identical in every lane after the reductions; made explicitly uniform so the
    // row loop stays a uniform loop (its queue step needs the whole wave).  A pivot that is
    // not positive (NaN included: fminf skips NaNs) fails on its own.
    const bool nonpos = __ballot(real && !(mypiv > 0.f)) != 0;
    const int bad = __builtin_amdgcn_readfirstlane((nonpos || !(pmin > 0.f) || (pmin < tau * dmax)) ? 1 : 0);
    if (bad) return false;
    // w = D^-1 L^-1 g, then L^T x = w from the last column: x_k = w_k once every later column
    // has been applied, then w_i += (-L_ki) x_k for i < k (lane i reads row k of the panel
    // that holds column i; lanes whose panel comes after row k read column 15 of panel K's
    // diagonal tile, which is zero in every row: the stored panels hold zeros on and above
    // the diagonal).
    float wv = g * __builtin_amdgcn_rcpf(mypiv);
    const int pk = ln >> 4;
    const int pbase = panel_row0<NT>(pk < NT ? pk : 0) - 16 * pk;
#pragma unroll
    for (int K = NT - 1; K >= 0; --K) {
        const bool ok = (pk <= K) && (ln < B);
        const float* rowp = ok ? pan + (pbase + 16 * K) * kPN + (ln & 15) : pan + panel_row0<NT>(K) * kPN + 15;
        float lt[16];
#pragma unroll
        for (int jj = 0; jj < 16; ++jj) lt[jj] = rowp[jj * kPN];
#pragma unroll
        for (int jj = 15; jj >= 0; --jj) wv = fmaf(lt[jj], readlane(wv, 16 * K + jj), wv);
        __builtin_amdgcn_sched_barrier(0);
    }
    wave_lds_fence();
    x = wv;
    return true;
}

template <int NT, bool FULL, bool TRANS, bool STATIC, bool BF, bool CF>
__global__ __launch_bounds__(256, 4) void k_sweep_rows(SweepArgs A) {
    constexpr int B = 16 * NT, NTL = ntiles<NT>();
    extern __shared__ float lds_all[];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, q16 = lane & 15, g4 = lane >> 4;
    float* pan = lds_all + wave * rows_lds_floats_per_wave<NT>();
    const int my_col = colmap<NT, FULL>(lane < B ? lane : 0);

    // STATIC: rows are dealt round-robin in the length order (sides whose rows are all
    // short); otherwise each wavefront takes the next row from a shared queue.
    int it = STATIC ? blockIdx.x * 4 + wave : 0;
    for (;;) {
        if constexpr (!STATIC) it = queue_next(&A.cursors[CUR_ROWS], lane);
        if (it >= A.nrows) break;
        const int r = A.order[it];
        if constexpr (STATIC) it += gridDim.x * 4;
        const int64_t lo = A.ptr[r], hi = A.ptr[r + 1];
        floatx4 acc[NTL];
#pragma unroll
        for (int id = 0; id < NTL; ++id) acc[id] = *reinterpret_cast<const floatx4*>(A.dtiles + id * 256 + lane * 4);
        float gp[NT];
#pragma unroll
        for (int t = 0; t < NT; ++t) gp[t] = 0.f;
        const int sf = A.seg_first[r];
        if (sf < 0) {
            float own[NT], ownc[TRANS ? NT : 1];
            load_own<NT, FULL, TRANS>(A, r, q16, own, ownc);
            accumulate<NT, FULL, TRANS, BF, kBatchSteps<TRANS, BF>, CF>(A, lo, hi, own, ownc, acc, gp, lane);
#pragma unroll
            for (int t = 0; t < NT; ++t) {
                gp[t] += __shfl_xor(gp[t], 16);
                gp[t] += __shfl_xor(gp[t], 32);
            }
        } else {
            const int ns = (int)((hi - lo + A.seg_len - 1) / A.seg_len);
            for (int s = sf; s < sf + ns; s += A.seg_group) {
                // the whole partial is loaded before it is added, so its loads are in flight together
                const float* P = A.seg_part + (size_t)s * seg_stride<NT>();
                floatx4 part[NTL];
                float pg[NT];
#pragma unroll
                for (int id = 0; id < NTL; ++id)
                    part[id] = __builtin_nontemporal_load(reinterpret_cast<const floatx4*>(P + ((size_t)id * 64 + lane) * 4));
#pragma unroll
                for (int t = 0; t < NT; ++t) pg[t] = __builtin_nontemporal_load(P + NTL * 256 + 16 * t + q16);
#pragma unroll
                for (int id = 0; id < NTL; ++id) acc[id] += part[id];
#pragma unroll
                for (int t = 0; t < NT; ++t) gp[t] += pg[t];
            }
        }
        // The lane id is laundered once per row so that the lane-dependent values below
        // are formed inside the row, not hoisted out of the row loop into registers.
        int ln = lane;
        asm volatile("" : "+v"(ln));
        const int my_col = colmap<NT, FULL>(ln < B ? ln : 0);
        // lane p < B holds the gradient entry of position p
        float g = 0.f;
#pragma unroll
        for (int t = 0; t < NT; ++t)
            if (g4 == t) g = gp[t];
        if (lane < B) g += A.R0[(size_t)r * B + my_col];
        float w;
        if (!ldl_solve<NT, FULL>(acc, g, pan, ln, A.tau, my_col, A.bw, w)) {
            // a pivot was rejected: the row is redone in float64
            if (lane == 0) {
                const int pos = atomicAdd(&A.cursors[CUR_FB_LIST], 1);
                A.fb_list[pos] = r;
            }
            continue;
        }
        // w (lane p) = delta at block column colmap(p)
        if (lane < B && my_col < A.bw) A.X[(size_t)r * A.d + A.p0 + my_col] -= w;
    }
}

// ---- Blocks of 65..128 coordinates (B = 128, NT = 8): one wavefront per row ----
//
// The 36 lower tiles of the Hessian stay in the wavefront's registers from the accumulation
// (accumulate<> as in the narrow kernel, lane q16 holding 8 block columns) to the back
// substitution; no other wavefront takes part in a row, so nothing waits on a workgroup
// barrier.  The LDL^T factorisation goes panel by panel: the panel's 16 columns pass through
// LDS to a lane-per-row layout relative to the panel (lane i holds panel row i and, for the
// first four panels, panel row 64 + i), are eliminated with the DPP steps of the narrow
// kernel (the forward substitution folded in), and return as -L into the same registers; the
// trailing tiles take A_IJ -= L_IK diag(piv) L_JK^T on the matrix cores.  The back
// substitution applies the off-diagonal -L tiles to the solved coordinates with matrix-core
// products (column 0 of the product) and solves each 16 x 16 unit triangle from a copy of its
// diagonal tile kept in LDS.
struct W8Lds {
    static constexpr int PAN = 0;               // the current panel: 128 rows at pitch kPS
    static constexpr int DT = PAN + 128 * kPS;  // the 8 diagonal tiles of -L, 16 x 16 row-major
    static constexpr int GL = DT + 8 * 256;     // [128] gradient, then z = L^-1 g
    static constexpr int PV = GL + 128;         // [128] pivots
    static constexpr int XS = PV + 128;         // [128] w = D^-1 z, then the solution
    static constexpr int YS = XS + 128;         // [16] off-diagonal sums of one tile row
    static constexpr int PER_WAVE = YS + 16;
};

// Steps KK..15 of panel K of the 128-wide LDL^T, with the look-ahead of panel_steps: piv and
// D (the pivot column of the panel's first row group, copied to every row group) were read
// for this step by the previous one.
template <int K, int KK>
__device__ __forceinline__ void w8_steps(float* p1, float* p2, float& g1, float& g2, float* pvl, float li, int src,
                                bool lead, float piv, float D) {
    if constexpr (KK < 16) {
        if (lead) pvl[16 * K + KK] = piv;
        const float nr = __builtin_amdgcn_rcpf(-piv);
        const float act = __builtin_amdgcn_fmed3f(li - (float)KK, 0.f, 1.f);  // 1 for the rows below KK
        const float tn1 = p1[KK] * nr * act;                                 // -t_i
        const float tn2 = K < 4 ? p2[KK] * nr : 0.f;                          // set 2: all below
        float pivn = 0.f, Dn = 0.f;
        if constexpr (KK < 15) {
            fmac_rowbcast<KK + 1, true>(p1[KK + 1], D, tn1);
            pivn = readlane(p1[KK + 1], KK + 1);
            if constexpr (KK < 14) Dn = __int_as_float(__builtin_amdgcn_ds_bpermute(src, __float_as_int(p1[KK + 1])));
            __builtin_amdgcn_sched_barrier(0);
            eliminate_cols<KK + 2, false>(p1, D, tn1);
            if constexpr (K < 4) eliminate_cols<KK + 1, true>(p2, D, tn2);
        }
        const float gk = readlane(g1, KK);
        g1 = fmaf(tn1, gk, g1);
        p1[KK] = tn1;
        if constexpr (K < 4) {
            g2 = fmaf(tn2, gk, g2);
            p2[KK] = tn2;
        }
        w8_steps<K, KK + 1>(p1, p2, g1, g2, pvl, li, src, lead, pivn, Dn);
    }
}

// Panel K of the 128-wide LDL^T (see above); lds: this wavefront's W8Lds region.
template <int K>
__device__ __forceinline__ void w8_panels(floatx4* acc, float* lds, int lane) {
    if constexpr (K < 8) {
        const int q16 = lane & 15, g4 = lane >> 4;
        float* PK = lds + W8Lds::PAN;
        float* GL = lds + W8Lds::GL;
        float* PV = lds + W8Lds::PV;
        constexpr int NR = 128 - 16 * K;  // rows of the panel
        // tiles (I, K) to LDS rows 16 (I - K) + row
#pragma unroll
        for (int I = K; I < 8; ++I) {
            const int id = I * (I + 1) / 2 + K;
#pragma unroll
            for (int j = 0; j < 4; ++j) PK[(16 * (I - K) + 4 * g4 + j) * kPS + q16] = acc[id][j];
        }
        wave_lds_fence();
        const bool v1 = lane < NR;
        const bool v2 = K < 4 && lane + 64 < NR;
        float p1[16], p2[16];
        const float* r1 = PK + (v1 ? lane : 0) * kPS;
        const float* r2 = PK + (v2 ? lane + 64 : 0) * kPS;
#pragma unroll
        for (int c4 = 0; c4 < 4; ++c4) {
            const float4 a = *reinterpret_cast<const float4*>(r1 + 4 * c4);
            p1[4 * c4 + 0] = v1 ? a.x : 0.f;
            p1[4 * c4 + 1] = v1 ? a.y : 0.f;
            p1[4 * c4 + 2] = v1 ? a.z : 0.f;
            p1[4 * c4 + 3] = v1 ? a.w : 0.f;
            if constexpr (K < 4) {
                const float4 b = *reinterpret_cast<const float4*>(r2 + 4 * c4);
                p2[4 * c4 + 0] = v2 ? b.x : 0.f;
                p2[4 * c4 + 1] = v2 ? b.y : 0.f;
                p2[4 * c4 + 2] = v2 ? b.z : 0.f;
                p2[4 * c4 + 3] = v2 ? b.w : 0.f;
            } else {
#pragma unroll
                for (int c = 0; c < 4; ++c) p2[4 * c4 + c] = 0.f;
            }
        }
        float g1 = v1 ? GL[16 * K + lane] : 0.f;
        float g2 = v2 ? GL[16 * K + 64 + lane] : 0.f;
        wave_lds_fence();
        {
            const int src = (lane & 15) * 4;
            const float piv0 = readlane(p1[0], 0);
            const float D0 = __int_as_float(__builtin_amdgcn_ds_bpermute(src, __float_as_int(p1[0])));
            w8_steps<K, 0>(p1, p2, g1, g2, PV, v1 ? (float)lane : -1.f, src, lane == 0, piv0, D0);
        }
        // the panel as -L (zeros on and above the diagonal), the updated gradient, and a copy
        // of the diagonal tile for the back substitution
        if (v1) {
#pragma unroll
            for (int c4 = 0; c4 < 4; ++c4)
                *reinterpret_cast<float4*>(PK + lane * kPS + 4 * c4) =
                    make_float4(p1[4 * c4], p1[4 * c4 + 1], p1[4 * c4 + 2], p1[4 * c4 + 3]);
            GL[16 * K + lane] = g1;
        }
        if (v2) {
#pragma unroll
            for (int c4 = 0; c4 < 4; ++c4)
                *reinterpret_cast<float4*>(PK + (lane + 64) * kPS + 4 * c4) =
                    make_float4(p2[4 * c4], p2[4 * c4 + 1], p2[4 * c4 + 2], p2[4 * c4 + 3]);
            GL[16 * K + 64 + lane] = g2;
        }
        if (lane < 16) {
            float* dt = lds + W8Lds::DT + K * 256 + lane * 16;
#pragma unroll
            for (int c4 = 0; c4 < 4; ++c4)
                *reinterpret_cast<float4*>(dt + 4 * c4) =
                    make_float4(p1[4 * c4], p1[4 * c4 + 1], p1[4 * c4 + 2], p1[4 * c4 + 3]);
        }
        wave_lds_fence();
        // -L_IK (I > K) back into the registers of tile (I, K) for the back substitution
#pragma unroll
        for (int I = K + 1; I < 8; ++I) {
            const int id = I * (I + 1) / 2 + K;
#pragma unroll
            for (int j = 0; j < 4; ++j) acc[id][j] = PK[(16 * (I - K) + 4 * g4 + j) * kPS + q16];
        }
        // trailing tiles: A_IJ -= L_IK diag(piv) L_JK^T for K < J <= I (the panel holds -L)
        if constexpr (K + 1 < 8) {
#pragma unroll
            for (int s4 = 0; s4 < 4; ++s4) {
                const float npm = -PV[16 * K + 4 * s4 + g4];
                float op[8];
#pragma unroll
                for (int I = K + 1; I < 8; ++I) op[I] = PK[(16 * (I - K) + q16) * kPS + 4 * s4 + g4];
#pragma unroll
                for (int I = K + 1; I < 8; ++I) {
                    const float a = op[I] * npm;
#pragma unroll
                    for (int J = K + 1; J <= I; ++J) {
                        const int id = I * (I + 1) / 2 + J;
                        acc[id] = mfma4(a, op[J], acc[id]);
                    }
                }
            }
        }
        wave_lds_fence();
        __builtin_amdgcn_sched_barrier(0);
        w8_panels<K + 1>(acc, lds, lane);
    }
}

// Back substitution for tile row K (from the last): x_K solves L_KK^T x_K = w_K - sum_{I>K}
// L_IK^T x_I, with -L_IK in the registers of tile (I, K) and -L_KK in LDS.
template <int K>
__device__ __forceinline__ void w8_back(const floatx4* acc, float* lds, int lane) {
    if constexpr (K >= 0) {
        const int q16 = lane & 15, g4 = lane >> 4;
        float* XS = lds + W8Lds::XS;
        float* YS = lds + W8Lds::YS;
        floatx4 y = floatx4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int I = K + 1; I < 8; ++I) {
            const int id = I * (I + 1) / 2 + K;
#pragma unroll
            for (int s = 0; s < 4; ++s) {
                const float b = q16 == 0 ? XS[16 * I + 4 * g4 + s] : 0.f;
                y = mfma4(acc[id][s], b, y);
            }
        }
        if constexpr (K < 7) {
            if (q16 == 0) {
#pragma unroll
                for (int j = 0; j < 4; ++j) YS[4 * g4 + j] = y[j];
            }
        }
        wave_lds_fence();
        const int i = lane & 15;
        float r = XS[16 * K + i] + (K < 7 ? YS[i] : 0.f);
        const float* dt = lds + W8Lds::DT + K * 256;
        float mc[16];
#pragma unroll
        for (int k = 0; k < 16; ++k) mc[k] = dt[k * 16 + i];  // -L_KK(k, i)
#pragma unroll
        for (int k = 15; k >= 0; --k) r = fmaf(mc[k], readlane(r, k), r);
        wave_lds_fence();
        if (lane < 16) XS[16 * K + lane] = r;
        wave_lds_fence();
        w8_back<K - 1>(acc, lds, lane);
    }
}

template <bool FULL, bool TRANS, bool BF, bool CF>
__global__ __launch_bounds__(256, 2) void k_rows_w8(SweepArgs A) {
    constexpr int NT = 8, B = 128, NTL = 36;
    extern __shared__ float lds_w8[];
    const int wave = threadIdx.x >> 6, lane0 = threadIdx.x & 63;
    float* lds = lds_w8 + wave * W8Lds::PER_WAVE;
    for (int it = blockIdx.x * 4 + wave; it < A.nrows; it += gridDim.x * 4) {
        const int r = A.order[it];
        const int64_t lo = A.ptr[r], hi = A.ptr[r + 1];
        int lane = lane0;  // laundered per row (see k_sweep_rows)
        asm volatile("" : "+v"(lane));
        const int q16 = lane & 15, g4 = lane >> 4;
        floatx4 acc[NTL];
#pragma unroll
        for (int id = 0; id < NTL; ++id) acc[id] = *reinterpret_cast<const floatx4*>(A.dtiles + id * 256 + lane * 4);
        float gp[NT];
#pragma unroll
        for (int t = 0; t < NT; ++t) gp[t] = 0.f;
        const int sf = A.seg_first[r];
        if (sf < 0) {
            float own[NT], ownc[TRANS ? NT : 1];
            load_own<NT, FULL, TRANS>(A, r, q16, own, ownc);
            accumulate<NT, FULL, TRANS, BF, 2, CF>(A, lo, hi, own, ownc, acc, gp, lane);
#pragma unroll
            for (int t = 0; t < NT; ++t) {
                gp[t] += __shfl_xor(gp[t], 16);
                gp[t] += __shfl_xor(gp[t], 32);
            }
        } else {
            const int ns = (int)((hi - lo + A.seg_len - 1) / A.seg_len);
            for (int s = sf; s < sf + ns; s += A.seg_group) {
                const float* P = A.seg_part + (size_t)s * seg_stride<NT>();
                // six tiles' loads in flight at a time (all 36 at once would need 144 more registers)
#pragma unroll
                for (int id0 = 0; id0 < NTL; id0 += 6) {
                    floatx4 part[6];
#pragma unroll
                    for (int u = 0; u < 6; ++u)
                        part[u] = __builtin_nontemporal_load(
                            reinterpret_cast<const floatx4*>(P + ((size_t)(id0 + u) * 64 + lane) * 4));
#pragma unroll
                    for (int u = 0; u < 6; ++u) acc[id0 + u] += part[u];
                    __builtin_amdgcn_sched_barrier(0);
                }
                if (g4 == 0) {
#pragma unroll
                    for (int t = 0; t < NT; ++t) gp[t] += __builtin_nontemporal_load(P + NTL * 256 + 16 * t + q16);
                }
            }
        }
        float* GL = lds + W8Lds::GL;
        if (g4 == 0) {
#pragma unroll
            for (int t = 0; t < NT; ++t)
                GL[16 * t + q16] = gp[t] + A.R0[(size_t)r * B + colmap<NT, FULL>(16 * t + q16)];
        }
        wave_lds_fence();
        const float dmax = diag_max<NT, FULL>(acc, lane, A.bw);
        w8_panels<0>(acc, lds, lane);
        // pivot check over the real (unpadded) coordinates, against the largest diagonal entry
        // (see ldl_solve)
        const float* PV = lds + W8Lds::PV;
        const float pa = PV[lane], pb = PV[64 + lane];
        const bool ra = colmap<NT, FULL>(lane) < A.bw, rb = colmap<NT, FULL>(64 + lane) < A.bw;
        float pmin = fminf(ra ? pa : 3.0e38f, rb ? pb : 3.0e38f);
#pragma unroll
        for (int m = 1; m < 64; m <<= 1) pmin = fminf(pmin, __shfl_xor(pmin, m));
        const bool nonpos = __ballot((ra && !(pa > 0.f)) || (rb && !(pb > 0.f))) != 0;
        const int bad = __builtin_amdgcn_readfirstlane((nonpos || !(pmin > 0.f) || (pmin < A.tau * dmax)) ? 1 : 0);
        if (bad) {
            if (lane == 0) {
                const int pos = atomicAdd(&A.cursors[CUR_FB_LIST], 1);
                A.fb_list[pos] = r;
            }
            continue;
        }
        float* XS = lds + W8Lds::XS;
        XS[lane] = GL[lane] * __builtin_amdgcn_rcpf(pa);
        XS[64 + lane] = GL[64 + lane] * __builtin_amdgcn_rcpf(pb);
        wave_lds_fence();
        w8_back<7>(acc, lds, lane);
        const float xa = XS[lane], xb = XS[64 + lane];
        const int ca = colmap<NT, FULL>(lane), cb = colmap<NT, FULL>(64 + lane);
        if (ca < A.bw) A.X[(size_t)r * A.d + A.p0 + ca] -= xa;
        if (cb < A.bw) A.X[(size_t)r * A.d + A.p0 + cb] -= xb;
        wave_lds_fence();
    }
}

// Float64 redo of rows whose float32 factorisation was rejected: the Hessian and
// gradient are re-accumulated from the gathered rows in float64 (with the cache
// already moved to this block by the pass), factored and solved in float64, and
// the row is updated.
template <int NT>
__global__ __launch_bounds__(256) void k_sweep_fallback(SweepArgs A) {
    constexpr int B = 16 * NT;
    constexpr int CH = 32;
    __shared__ double Hm[B][B + 1];
    __shared__ double xs[CH][B];
    __shared__ double gv[B], own[B];
    __shared__ double rs[CH], ws[CH];
    __shared__ int ok;
    const int tid = threadIdx.x;
    const int nfb = A.cursors[CUR_FB_LIST];
    for (int idx = blockIdx.x; idx < nfb; idx += gridDim.x) {
        const int r = A.fb_list[idx];
        const int64_t lo = A.ptr[r], hi = A.ptr[r + 1];
        for (int e = tid; e < B * B; e += 256) Hm[e / B][e % B] = (double)A.Dmat[e];
        if (tid < B) {
            gv[tid] = (double)A.R0[(size_t)r * B + tid];
            own[tid] = tid < A.bw ? (double)A.X[(size_t)r * A.d + A.p0 + tid] : 0.0;
        }
        if (tid == 0) ok = 1;
        __syncthreads();
        for (int64_t c0 = lo; c0 < hi; c0 += CH) {
            for (int e = tid; e < CH * B; e += 256) {
                const int j = e / B, c = e % B;
                const int64_t k = c0 + j;
                xs[j][c] = (k < hi && c < A.bw) ? (double)A.Xo[(size_t)A.col[k] * A.d + A.p0 + c] : 0.0;
            }
            __syncthreads();
            if (tid < CH) {
                const int64_t k = c0 + tid;
                double res = 0.0, w = 0.0;
                if (k < hi) {
                    const int64_t s = A.slot ? (int64_t)A.slot[k] : k;
                    const double ak = A.a ? (double)A.a[k] : 1.0;
                    const double yk = A.y ? (double)A.y[k] : 1.0;
                    double yh = (double)A.cache[s];
                    for (int c = 0; c < A.bw; ++c) yh += own[c] * xs[tid][c];
                    res = ak * (yh - yk);
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
        __syncthreads();
    }
}

template <int NT, bool FULL, bool TRANS, bool BF, bool CF>
void launch_sweep_nt_cf(ials_ctx* c, const SweepArgs& args, const SideIndex& s, int sd) {
    hipStream_t st = c->stream;
    const unsigned max_blocks = (unsigned)c->num_cu * 8;
    if (s.nseg > 0) {
        ProfScope ps(c, IALS_K_SEG_USER + sd);
        hipLaunchKernelGGL((k_sweep_seg<NT, FULL, TRANS, BF, CF>), dim3(std::min<unsigned>(max_blocks, (s.nseg + 3) / 4)),
                           dim3(256), 0, st, args);
        launch_seg_group(st, args, seg_stride<NT>());
    }
    if (s.nrows > 0) {
        const size_t lds = sizeof(float) * rows_lds_floats<NT>();
        hipLaunchKernelGGL((k_make_dtiles<NT, FULL>), dim3((ntiles<NT>() * 256 + 255) / 256), dim3(256), 0, st, args.Dmat,
                           args.dtiles);
        {
            ProfScope ps(c, (TRANS ? IALS_K_ROWS_USER_MOVE : IALS_K_ROWS_USER) + sd);
            if (args.rows_batch == 0) {
                // static dealing: exactly the blocks that are resident at once
                static OccCache occ;
                const int resident = resident_per_cu(
                    occ, reinterpret_cast<const void*>(&k_sweep_rows<NT, FULL, TRANS, true, BF, CF>), 256, lds, false, 2);
                hipLaunchKernelGGL((k_sweep_rows<NT, FULL, TRANS, true, BF, CF>),
                                   dim3(std::min<unsigned>((unsigned)(c->num_cu * resident), (s.nrows + 3) / 4)),
                                   dim3(256), lds, st, args);
            } else {
                hipLaunchKernelGGL((k_sweep_rows<NT, FULL, TRANS, false, BF, CF>),
                                   dim3(std::min<unsigned>(max_blocks, (s.nrows + 3) / 4)), dim3(256), lds, st, args);
            }
        }
        ProfScope ps(c, IALS_K_FALLBACK_USER + sd);
        hipLaunchKernelGGL((k_sweep_fallback<NT>), dim3((unsigned)c->num_cu), dim3(256), 0, st, args);
    }
}

// the passes that move the cache come in two forms, by whether the cache's block is full
template <int NT, bool FULL, bool TRANS, bool BF>
void launch_sweep_nt(ials_ctx* c, const SweepArgs& args, const SideIndex& s, int sd) {
    if constexpr (TRANS) {
        if (!args.cur_full) {
            launch_sweep_nt_cf<NT, FULL, TRANS, BF, false>(c, args, s, sd);
            return;
        }
    }
    launch_sweep_nt_cf<NT, FULL, TRANS, BF, true>(c, args, s, sd);
}

template <int NT>
bool vec_ok(const SweepArgs& A, int p0, int bw, const float* X) {
    constexpr int B = 16 * NT;
    if (NT == 3) return false;
    return bw == B && (A.d % NT == 0) && (p0 % NT == 0) && ((reinterpret_cast<uintptr_t>(X) % (4 * NT)) == 0);
}

template <int NT, bool BF>
void launch_sweep_b(ials_ctx* c, SweepArgs& A, const SideIndex& s, int sd, bool trans) {
    const bool full = vec_ok<NT>(A, A.p0, A.bw, A.Xo) && vec_ok<NT>(A, A.p0, A.bw, A.X);
    A.cur_full = vec_ok<NT>(A, A.pc, A.bwc, A.Xo) && vec_ok<NT>(A, A.pc, A.bwc, A.X);
    if (full) {
        if (trans)
            launch_sweep_nt<NT, true, true, BF>(c, A, s, sd);
        else
            launch_sweep_nt<NT, true, false, BF>(c, A, s, sd);
    } else {
        if (trans)
            launch_sweep_nt<NT, false, true, BF>(c, A, s, sd);
        else
            launch_sweep_nt<NT, false, false, BF>(c, A, s, sd);
    }
}

template <bool BF>
void launch_sweep_prec(ials_ctx* c, SweepArgs& A, const SideIndex& s, int sd, bool trans) {
    switch (c->B) {
        case 16: launch_sweep_b<1, BF>(c, A, s, sd, trans); break;
        case 32: launch_sweep_b<2, BF>(c, A, s, sd, trans); break;
        case 48: launch_sweep_b<3, BF>(c, A, s, sd, trans); break;
        default: launch_sweep_b<4, BF>(c, A, s, sd, trans); break;
    }
}

template <bool FULL, bool TRANS, bool BF, bool CF>
void launch_w8_nt_cf(ials_ctx* c, const SweepArgs& args, const SideIndex& s, int sd) {
    hipStream_t st = c->stream;
    const unsigned max_blocks = (unsigned)c->num_cu * 8;
    if (s.nseg > 0) {
        ProfScope ps(c, IALS_K_SEG_USER + sd);
        hipLaunchKernelGGL((k_sweep_seg<8, FULL, TRANS, BF, CF>), dim3(std::min<unsigned>(max_blocks, (s.nseg + 3) / 4)),
                           dim3(256), 0, st, args);
        launch_seg_group(st, args, seg_stride<8>());
    }
    if (s.nrows > 0) {
        const size_t lds = sizeof(float) * 4 * W8Lds::PER_WAVE;
        hipLaunchKernelGGL((k_make_dtiles<8, FULL>), dim3((ntiles<8>() * 256 + 255) / 256), dim3(256), 0, st, args.Dmat,
                           args.dtiles);
        {
            ProfScope ps(c, (TRANS ? IALS_K_ROWS_USER_MOVE : IALS_K_ROWS_USER) + sd);
            // static dealing over exactly the workgroups that are resident at once
            static OccCache occ;
            const int resident =
                resident_per_cu(occ, reinterpret_cast<const void*>(&k_rows_w8<FULL, TRANS, BF, CF>), 256, lds, true, 1);
            hipLaunchKernelGGL((k_rows_w8<FULL, TRANS, BF, CF>),
                               dim3(std::min<unsigned>((unsigned)(c->num_cu * resident), (s.nrows + 3) / 4)),
                               dim3(256), lds, st, args);
        }
        ProfScope ps(c, IALS_K_FALLBACK_USER + sd);
        launch_fallback_big(c, args);
    }
}

template <bool FULL, bool TRANS, bool BF>
void launch_w8_nt(ials_ctx* c, const SweepArgs& args, const SideIndex& s, int sd) {
    if constexpr (TRANS) {
        if (!args.cur_full) {
            launch_w8_nt_cf<FULL, TRANS, BF, false>(c, args, s, sd);
            return;
        }
    }
    launch_w8_nt_cf<FULL, TRANS, BF, true>(c, args, s, sd);
}

template <bool BF>
void launch_sweep_w8(ials_ctx* c, SweepArgs& A, const SideIndex& s, int sd, bool trans) {
    const bool full = vec_ok<8>(A, A.p0, A.bw, A.Xo) && vec_ok<8>(A, A.p0, A.bw, A.X);
    A.cur_full = vec_ok<8>(A, A.pc, A.bwc, A.Xo) && vec_ok<8>(A, A.pc, A.bwc, A.X);
    A.fb_scratch = c->fb_scratch;
    if (full) {
        if (trans)
            launch_w8_nt<true, true, BF>(c, A, s, sd);
        else
            launch_w8_nt<true, false, BF>(c, A, s, sd);
    } else {
        if (trans)
            launch_w8_nt<false, true, BF>(c, A, s, sd);
        else
            launch_w8_nt<false, false, BF>(c, A, s, sd);
    }
}

}  // namespace

void launch_seg_group(hipStream_t st, const SweepArgs& A, int32_t stride) {
    if (A.seg_group < 2 || A.nseg == 0) return;
    hipLaunchKernelGGL(k_seg_group, dim3((unsigned)A.nseg, (unsigned)((stride + 1023) / 1024)), dim3(256), 0, st, A,
                       stride);
}

size_t seg_part_floats_per_segment(int32_t B) {
    const int NT = B / 16;
    return (size_t)(NT * (NT + 1) / 2) * 256 + (size_t)B;
}

// One pass of block blk on side sd; the cache moves to blk if it is relative to another block.
void launch_sweep(ials_ctx* c, int sd, int32_t blk) {
    if (c->b == 1) {  // scalar coordinate descent: no padded block, no factorisation
        launch_icd_pass(c, sd, blk);
        return;
    }
    const SideIndex& s = c->side[sd];
    SweepArgs A;
    A.ptr = s.ptr;
    A.col = s.col;
    A.slot = s.slot;
    A.y = s.y;
    A.a = s.a;
    A.X = sd == IALS_SIDE_USER ? c->W : c->H;
    A.Xo = sd == IALS_SIDE_USER ? c->H : c->W;
    A.cache = c->yhat;
    A.R0 = c->R0;
    A.Dmat = c->Dmat;
    A.dtiles = c->dtiles;
    A.d = c->d;
    A.p0 = blk * c->b;
    A.bw = std::min(c->b, c->d - A.p0);
    A.pc = c->cur_block * c->b;
    A.bwc = std::min(c->b, c->d - A.pc);
    A.cur_full = 0;
    A.nrows = s.nrows;
    A.order = s.order;
    A.seg_first = s.seg_first;
    A.seg_row = s.seg_row;
    A.seg_lo = s.seg_lo;
    A.seg_hi = s.seg_hi;
    A.seg_order = s.seg_order;
    A.nseg = s.nseg;
    A.seg_part = c->seg_part;
    A.fb_list = c->fb_list;
    A.cursors = c->cursors;
    A.counters = c->counters;
    A.tau = c->tau;
    // static dealing unless asked otherwise: a row's work is bounded (rows longer than a
    // segment add a few group partials), and the queue's atomics cost more than its balance gains
    A.rows_batch = (c->flags & IALS_FLAG_DEAL_QUEUE) ? 1 : 0;
    A.seg_len = c->seg_len;
    // sqrt(ns) groups of sqrt(ns) segments for the longest row once it has more than 8 segments
    const int64_t max_ns = (s.max_len + c->seg_len - 1) / c->seg_len;
    A.seg_group = max_ns > 8 ? (int32_t)std::ceil(std::sqrt((double)max_ns)) : 1;
    const bool trans = blk != c->cur_block;
    if (c->B == 128) {  // one wavefront per row
        if (c->precision == IALS_PREC_BF16)
            launch_sweep_w8<true>(c, A, s, sd, trans);
        else
            launch_sweep_w8<false>(c, A, s, sd, trans);
    } else if (c->B > 64)
        launch_sweep_big(c, A, s, sd, trans);
    else if (c->precision == IALS_PREC_BF16)
        launch_sweep_prec<true>(c, A, s, sd, trans);
    else
        launch_sweep_prec<false>(c, A, s, sd, trans);
    c->cur_block = blk;
}

}  // namespace ials
