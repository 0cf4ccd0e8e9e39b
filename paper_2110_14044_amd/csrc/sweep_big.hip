// The block pass of iALS++ (sec. 4, eq. 8-9, Alg. 3) for blocks wider than 64
// coordinates: B = 128 (NT = 8 tiles of 16) or B = 256 (NT = 16).
//
// One workgroup of NT/2 wavefronts per row.  Wave w owns the lower tiles of the
// two tile rows w and NT-1-w (NT+1 tiles, the same count for every wave).
//
// Accumulation: every wave walks the row's observations; per observation it
// gathers the partner's block (lane q16 of group g4 takes columns 16t + q16),
// forms the prediction from the cache and the row's own block, and adds
// a_k x x^T into its own tiles on the matrix cores (float32 16x16x4 per four
// observations, or bfloat16 16x16x16 per sixteen).  Wave 0 also accumulates the
// gradient and moves the cache.  Rows longer than the segment length take
// per-segment partials instead (k_seg_big), summed in segment order.
//
// Factorisation: the tiles go to LDS (packed lower tiles, 16 rows at a pitch of 20 floats,
// or 16 when B = 256) and a blocked right-looking LDL^T runs over them, panel by panel.  The 16 columns of panel K
// go to a lane per row: every wave holds the panel's diagonal tile in lanes 0-15 and its
// share of the rows below in the other lanes, and eliminates them step by step with the
// forward substitution folded in (column k of the diagonal tile is copied to every 16-lane
// row and read with a DPP row broadcast, so each update is one fused multiply-add); the
// panel goes back as -L with the pivots, and after a barrier every wave subtracts
// L_IK diag(piv) L_JK^T from its own tiles (I, J), K < J <= I, on the matrix cores.  Wave 0
// then solves L^T x = D^-1 z column by column from the last.  A row whose pivots fail the
// ratio test is redone in float64 by k_fallback_big.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "ials_internal.h"

namespace ials {
namespace {

__device__ inline floatx4 mfma4(float a, float b, floatx4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
__device__ inline floatx4 mfma_bf16(shortx4 a, shortx4 b, floatx4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
}
__device__ inline short bf16s(float f) {
    const unsigned u = __float_as_uint(f);
    return (short)((u + 0x7fffu + ((u >> 16) & 1u)) >> 16);
}
__device__ inline float readlane(float x, int l) {
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x), l));
}
__device__ inline float sum16(float s) { return row_sum16(s); }
__device__ inline void wave_fence() {
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
    __builtin_amdgcn_wave_barrier();
}
__device__ inline int tile_id(int I, int J) { return I * (I + 1) / 2 + J; }

template <int NT>
struct BigLds {
    static constexpr int B = 16 * NT, NW = NT / 2, NTL = NT * (NT + 1) / 2;
    // row pitch of a tile in LDS: 20 floats spread the accesses over the banks (rows stay
    // 16-byte aligned); B = 256 keeps 16 for its LDS budget
    static constexpr int TP = NT <= 8 ? 20 : 16, TSZ = 16 * TP;
    static constexpr int MAT = 0;                 // NTL packed lower tiles, row-major 16 x 16 at pitch TP
    static constexpr int YP = MAT + NTL * TSZ;    // [TSZ] a zero tile, then [B] the pivots
    static constexpr int XW = YP + TSZ + B;       // [NW][B]   each wave's copy of the solution
    static constexpr int G = XW + NW * B;         // [B]       gradient, then z = L^-1 g
    static constexpr int SP = G + B;              // [2][NW][16] back-substitution partials
    static constexpr int OWN = SP + 2 * NW * 16;  // [2][B] the row's own values (pass block, cache block)
    static constexpr int DM = OWN + 2 * B;        // [NW] each wave's largest diagonal entry
    static constexpr int TOTAL = DM + NW;
};

// x[t] = X[i][p0 + 16t + q16] (0 outside the block)
template <int NT>
__device__ inline void load_block(const float* __restrict__ X, int d, int i, int p0, int bw, int q16, float* x) {
    const float* xr = X + (size_t)i * d + p0;
#pragma unroll
    for (int t = 0; t < NT; ++t) {
        const int c = 16 * t + q16;
        const float v = xr[c < bw ? c : 0];
        x[t] = c < bw ? v : 0.f;
    }
}
template <int NT>
__device__ inline float pick(const float* x, int I) {
    float r = 0.f;
#pragma unroll
    for (int t = 0; t < NT; ++t) r = (t == I) ? x[t] : r;
    return r;
}

// The wave's NT+1 tiles: m <= I1 is tile (I1, m); m > I1 is tile (I2, m - I1 - 1), I2 = NT-1-I1.
__device__ inline void tile_of(int m, int I1, int NT, int& I, int& J) {
    if (m <= I1) {
        I = I1;
        J = m;
    } else {
        I = NT - 1 - I1;
        J = m - I1 - 1;
    }
}

// own / ownc: the row's values at this pass's block and at the cache's block (LDS, by column).
// acc[m] (the wave's tiles) += sum_k a_k x_k x_k^T over observations [lo, hi); the lead
// wave also accumulates gp[t] += sum_k a_k (yhat_k - y_k) x_k[t] and, with TRANS, moves
// the cache entries to this pass's block.  The gathered values go through this wave's
// LDS staging area (NT x 64 floats, or NT x 64 packed bfloat16 quadruples) so that a
// tile's column operand is addressed by its index.
// Steps of 4 observations per batch of partner-row loads (registers: UB x NT x (1 + TRANS)).
template <int NT, bool TRANS>
constexpr int kBigBatch = NT == 8 ? (TRANS ? 2 : 4) : 1;

template <int NT, bool TRANS, bool BF, int UB = kBigBatch<NT, TRANS>>
__device__ void big_accumulate(const SweepArgs& A, int64_t lo, int64_t hi, const float* own, const float* ownc,
                               int I1, floatx4* acc, float* gp, bool lead, int lane, float* stage) {
    const int q16 = lane & 15, g4 = lane >> 4;
    const int I2 = NT - 1 - I1;
    for (int64_t c0 = lo; c0 < hi; c0 += 64) {
        const int64_t k = c0 + lane;
        const bool v = k < hi;
        int ci = 0, si = 0;
        float cv = 0.f, yv = 1.f, av = 1.f;
        if (v) {
            ci = A.col[k];
            si = A.slot ? A.slot[k] : (int)k;
            cv = A.cache[si];
            if (A.y) yv = A.y[k];
            if (A.a) av = A.a[k];
        }
        const int cnt = (int)std::min<int64_t>(64, hi - c0);
        const int nsteps = (cnt + 3) >> 2;
        for (int st = 0; st < nsteps; st += 4) {
            shortx4 pa1{0, 0, 0, 0}, pa2{0, 0, 0, 0}, pb[BF ? NT : 1];
            if constexpr (BF) {
#pragma unroll
                for (int t = 0; t < NT; ++t) pb[t] = shortx4{0, 0, 0, 0};
            }
            // UB steps at a time with all their partner rows loaded first; steps past the
            // chunk load a valid row and weigh 0 (no branches, so the loads are in flight together)
#pragma unroll
            for (int u0 = 0; u0 < 4; u0 += UB) {
                float xb[UB][NT], xcb[UB][TRANS ? NT : 1];
#pragma unroll
                for (int uu = 0; uu < UB; ++uu) {
                    const int i = __shfl(ci, (4 * (st + u0 + uu) + g4) & 63);
                    load_block<NT>(A.Xo, A.d, i, A.p0, A.bw, q16, xb[uu]);
                    if constexpr (TRANS) load_block<NT>(A.Xo, A.d, i, A.pc, A.bwc, q16, xcb[uu]);
                }
#pragma unroll
                for (int uu = 0; uu < UB; ++uu) {
                    const int u = u0 + uu;
                    const float* x = xb[uu];
                    const int src = 4 * (st + u) + g4;
                    const bool valid = src < cnt;
                    const float ck = __shfl(cv, src & 63);
                    const float yk = A.y ? __shfl(yv, src & 63) : 1.f;
                    const float ak_all = A.a ? __shfl(av, src & 63) : 1.f;
                    const float ak = valid ? ak_all : 0.f;
                    float sp = 0.f;
#pragma unroll
                    for (int t = 0; t < NT; ++t) sp = fmaf(x[t], own[16 * t + q16], sp);
                    sp = sum16(sp);
                    float yh = ck + sp;
                    if constexpr (TRANS) {
                        float sc = 0.f;
#pragma unroll
                        for (int t = 0; t < NT; ++t) sc = fmaf(xcb[uu][t], ownc[16 * t + q16], sc);
                        sc = sum16(sc);
                        yh = ck + sc;
                        const int sk = __shfl(si, src & 63);
                        if (lead && q16 == 0 && valid) A.cache[sk] = yh - sp;
                    }
                    const float rk = ak * (yh - yk);
                    if (lead) {
#pragma unroll
                        for (int t = 0; t < NT; ++t) gp[t] = fmaf(rk, x[t], gp[t]);
                    }
                    const float xa1 = ak * pick<NT>(x, I1);
                    const float xa2 = ak * pick<NT>(x, I2);
                    if constexpr (BF) {
                        pa1[u] = bf16s(xa1);
                        pa2[u] = bf16s(xa2);
#pragma unroll
                        for (int t = 0; t < NT; ++t) pb[t][u] = bf16s(x[t]);
                    } else {
#pragma unroll
                        for (int t = 0; t < NT; ++t) stage[t * 64 + lane] = x[t];
                        wave_fence();
#pragma unroll
                        for (int m = 0; m <= NT; ++m) {
                            const int J = m <= I1 ? m : m - I1 - 1;
                            acc[m] = mfma4(m <= I1 ? xa1 : xa2, stage[J * 64 + lane], acc[m]);
                        }
                        wave_fence();
                    }
                }
            }
            if constexpr (BF) {
                shortx4* st4 = reinterpret_cast<shortx4*>(stage);
#pragma unroll
                for (int t = 0; t < NT; ++t) st4[t * 64 + lane] = pb[t];
                wave_fence();
#pragma unroll
                for (int m = 0; m <= NT; ++m) {
                    const int J = m <= I1 ? m : m - I1 - 1;
                    acc[m] = mfma_bf16(m <= I1 ? pa1 : pa2, st4[J * 64 + lane], acc[m]);
                }
                wave_fence();
            }
        }
    }
}

// floats of one segment partial: NTL tiles in accumulator layout + B gradient entries
template <int NT>
constexpr int big_seg_stride() { return NT * (NT + 1) / 2 * 256 + 16 * NT; }

// the row's own block values (this pass's block and the cache's block) into LDS
template <int NT, bool TRANS>
__device__ inline void own_to_lds(const SweepArgs& A, int r, float* own, float* ownc) {
    constexpr int B = 16 * NT;
    for (int q = threadIdx.x; q < B; q += blockDim.x) {
        own[q] = q < A.bw ? A.X[(size_t)r * A.d + A.p0 + q] : 0.f;
        if constexpr (TRANS) ownc[q] = q < A.bwc ? A.X[(size_t)r * A.d + A.pc + q] : 0.f;
    }
}

template <int NT, bool TRANS, bool BF>
__global__ __launch_bounds__(NT * 32) void k_seg_big(SweepArgs A) {
    __shared__ __align__(16) float stage_all[NT / 2][NT * 128];
    __shared__ float own[16 * NT], ownc[16 * NT];
    const int lane = threadIdx.x & 63, q16 = lane & 15, g4 = lane >> 4;
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int I1 = wave;
    const bool lead = wave == 0;
    for (int it = blockIdx.x; it < A.nseg; it += gridDim.x) {
        floatx4 acc[NT + 1];
        float gp[NT];
#pragma unroll
        for (int m = 0; m <= NT; ++m) acc[m] = floatx4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int t = 0; t < NT; ++t) gp[t] = 0.f;
        const int r = A.seg_row[it];
        __syncthreads();  // the previous segment's readers are done with own / ownc
        own_to_lds<NT, TRANS>(A, r, own, ownc);
        __syncthreads();
        big_accumulate<NT, TRANS, BF>(A, A.seg_lo[it], A.seg_hi[it], own, ownc, I1, acc, gp, lead, lane,
                                      stage_all[wave]);
        float* P = A.seg_part + (size_t)it * big_seg_stride<NT>();
#pragma unroll
        for (int m = 0; m <= NT; ++m) {
            int I, J;
            tile_of(m, I1, NT, I, J);
            *reinterpret_cast<floatx4*>(P + ((size_t)tile_id(I, J) * 64 + lane) * 4) = acc[m];
        }
        if (lead) {
#pragma unroll
            for (int t = 0; t < NT; ++t) {
                gp[t] += __shfl_xor(gp[t], 16);
                gp[t] += __shfl_xor(gp[t], 32);
            }
            if (g4 == 0) {
#pragma unroll
                for (int t = 0; t < NT; ++t) P[NT * (NT + 1) / 2 * 256 + 16 * t + q16] = gp[t];
            }
        }
    }
}

// tile (accumulator layout: lane l, register j = element (4(l/16)+j, l%16)) <-> LDS row-major, pitch TP
template <int TP>
__device__ inline void tile_store(float* T, floatx4 c, int lane) {
#pragma unroll
    for (int j = 0; j < 4; ++j) T[(4 * (lane >> 4) + j) * TP + (lane & 15)] = c[j];
}
template <int TP>
__device__ inline floatx4 tile_load(const float* T, int lane) {
    floatx4 c;
#pragma unroll
    for (int j = 0; j < 4; ++j) c[j] = T[(4 * (lane >> 4) + j) * TP + (lane & 15)];
    return c;
}
// c -= (P diag(pv)) Q^T for 16 x 16 row-major tiles P, Q at pitch TP (pv: the 16 pivots of P's columns)
template <int TP>
__device__ inline floatx4 mm_pdqt(floatx4 c, const float* P, const float* Q, const float* pv, int lane) {
#pragma unroll
    for (int s = 0; s < 4; ++s) {
        const int o = (lane & 15) * TP + 4 * s + (lane >> 4);
        c = mfma4(-P[o] * pv[4 * s + (lane >> 4)], Q[o], c);
    }
    return c;
}

// Steps KK..15 of a panel with one row per lane: lanes 0-15 hold the panel's diagonal tile,
// the other lanes rows below it (see big_panel); lk = this lane's row - 16K (< 0: no row).
template <int KK>
__device__ inline void big_steps(float* p, float& g, float* pvl, float lk, int K, int src, bool lead) {
    if constexpr (KK < 16) {
        const float piv = readlane(p[KK], KK);
        if (lead) pvl[16 * K + KK] = piv;
        const float nr = __builtin_amdgcn_rcpf(-piv);
        const float tn = p[KK] * nr * __builtin_amdgcn_fmed3f(lk - (float)KK, 0.f, 1.f);  // -t_i
        if constexpr (KK < 15) {
            const float D = __int_as_float(__builtin_amdgcn_ds_bpermute(src, __float_as_int(p[KK])));
            eliminate_cols<KK + 1, true>(p, D, tn);
        }
        g = fmaf(tn, readlane(g, KK), g);
        p[KK] = tn;
        big_steps<KK + 1>(p, g, pvl, lk, K, src, lead);
    }
}

// Panel K of the LDL^T factorisation, shared by the NW wavefronts: every wave holds the
// panel's 16 x 16 diagonal tile in lanes 0-15 (the same rows, eliminated identically in
// every wave) and its share of the rows below in lanes 16-63 (NT <= 16 keeps a share within
// 48 rows).  Each step k takes piv = A_kk, t_i = A_ik / piv for the rows below k,
// g_i -= t_i g_k and A_ij -= t_i A_jk for the panel's later columns, column k of the
// diagonal tile being copied to every 16-lane row and read with a row broadcast.  A wave
// writes back its own rows (wave 0 also the diagonal tile and the pivots) holding -t, zeros
// on and above the diagonal; gl holds the gradient, updated in place.
template <int NT>
__device__ inline void big_panel(float* mat, float* pvl, float* gl, int lane, int wave, int K) {
    constexpr int B = 16 * NT, NW = NT / 2;
    const int below = B - 16 * K - 16;           // rows under the diagonal tile
    const int share = (below + NW - 1) / NW;    // rows per wave
    int r;
    if (lane < 16) {
        r = 16 * K + lane;
    } else {
        const int j = lane - 16;
        r = (j < share) ? 16 * K + 16 + wave * share + j : B;
        if (r >= B) r = -1;
    }
    const bool has = r >= 0;
    constexpr int TP = BigLds<NT>::TP, TSZ = BigLds<NT>::TSZ;
    const float* src = has ? mat + tile_id(r >> 4, K) * TSZ + (r & 15) * TP : mat;
    float p[16];
#pragma unroll
    for (int c4 = 0; c4 < 4; ++c4) {
        const float4 v = *reinterpret_cast<const float4*>(src + 4 * c4);
        p[4 * c4 + 0] = v.x;
        p[4 * c4 + 1] = v.y;
        p[4 * c4 + 2] = v.z;
        p[4 * c4 + 3] = v.w;
    }
    float g = has ? gl[r] : 0.f;
    const float lk = has ? (float)(r - 16 * K) : -1.f;
    __syncthreads();  // every wave has read the diagonal tile before wave 0 writes it back
    big_steps<0>(p, g, pvl, lk, K, (lane & 15) * 4, wave == 0 && lane == 0);
    // rows below the tile: their wave; the diagonal tile: wave 0 (every wave holds it)
    if (has && (lane >= 16 || wave == 0)) {
        float* dst = mat + tile_id(r >> 4, K) * TSZ + (r & 15) * TP;
#pragma unroll
        for (int c4 = 0; c4 < 4; ++c4)
            *reinterpret_cast<float4*>(dst + 4 * c4) = make_float4(p[4 * c4], p[4 * c4 + 1], p[4 * c4 + 2], p[4 * c4 + 3]);
        gl[r] = g;
    }
}

template <int NT, bool TRANS, bool BF>
__global__ __launch_bounds__(NT * 32) void k_rows_big(SweepArgs A) {
    using L = BigLds<NT>;
    constexpr int B = L::B, NTL = L::NTL, NH = B / 64;
    extern __shared__ __align__(16) float lds_big[];
    const int lane0 = threadIdx.x & 63;
    const int wave0 = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    static_assert(BigLds<NT>::NW * NT * 128 <= BigLds<NT>::NTL * BigLds<NT>::TSZ, "staging fits in the matrix region");
    constexpr int TP = L::TP, TSZ = L::TSZ;
    float* mat = lds_big + L::MAT;
    float* gl = lds_big + L::G;
    for (int e = threadIdx.x; e < TSZ; e += blockDim.x) lds_big[L::YP + e] = 0.f;
    __syncthreads();

    for (int it = blockIdx.x; it < A.nrows; it += gridDim.x) {
        const int r = A.order[it];
        const int64_t lo = A.ptr[r], hi = A.ptr[r + 1];
        // The lane and wave ids are laundered per row so that the row-invariant addresses
        // derived from them are formed inside the row, not hoisted out of the row loop
        // into registers for the whole kernel.
        int lane = lane0, I1 = wave0;
        asm volatile("" : "+v"(lane));
        asm volatile("" : "+s"(I1));
        const int q16 = lane & 15, g4 = lane >> 4, I2 = NT - 1 - I1;
        const bool lead = I1 == 0;
        floatx4 acc[NT + 1];
        float gp[NT];
        const float* Dm = A.Dmat;
        // the Hessian starts from alpha0 G_pipi + lambda I
#pragma unroll
        for (int m = 0; m <= NT; ++m) {
            int I, J;
            tile_of(m, I1, NT, I, J);
#pragma unroll
            for (int j = 0; j < 4; ++j) acc[m][j] = Dm[(size_t)(16 * I + 4 * g4 + j) * B + 16 * J + q16];
        }
#pragma unroll
        for (int t = 0; t < NT; ++t) gp[t] = 0.f;
        const int sf = A.seg_first[r];
        if (sf < 0) {
            float* own = lds_big + L::OWN;
            own_to_lds<NT, TRANS>(A, r, own, own + B);
            __syncthreads();
            // staging aliases the matrix region, which is not in use yet
            big_accumulate<NT, TRANS, BF>(A, lo, hi, own, own + B, I1, acc, gp, lead, lane, mat + I1 * NT * 128);
            if (lead) {
#pragma unroll
                for (int t = 0; t < NT; ++t) {
                    gp[t] += __shfl_xor(gp[t], 16);
                    gp[t] += __shfl_xor(gp[t], 32);
                }
            }
        } else {
            const int ns = (int)((hi - lo + A.seg_len - 1) / A.seg_len);
            for (int s = sf; s < sf + ns; s += A.seg_group) {
                // this wavefront's tiles of the partial are loaded before they are added
                const float* P = A.seg_part + (size_t)s * big_seg_stride<NT>();
                floatx4 part[NT + 1];
#pragma unroll
                for (int m = 0; m <= NT; ++m) {
                    int I, J;
                    tile_of(m, I1, NT, I, J);
                    part[m] = __builtin_nontemporal_load(
                        reinterpret_cast<const floatx4*>(P + ((size_t)tile_id(I, J) * 64 + lane) * 4));
                }
#pragma unroll
                for (int m = 0; m <= NT; ++m) acc[m] += part[m];
                if (lead) {
#pragma unroll
                    for (int t = 0; t < NT; ++t) gp[t] += P[NTL * 256 + 16 * t + q16];
                }
            }
        }
        if (lead && g4 == 0) {
#pragma unroll
            for (int t = 0; t < NT; ++t) gl[16 * t + q16] = gp[t] + A.R0[(size_t)r * B + 16 * t + q16];
        }
        {
            // largest diagonal entry over the real coordinates of this wave's diagonal tiles
            // (lane (q16, g4) holds row 4 g4 + j, column q16 of a tile)
            const int jd = q16 - 4 * g4;
            float dm = 0.f;
#pragma unroll
            for (int m = 0; m <= NT; ++m) {
                int I, J;
                tile_of(m, I1, NT, I, J);
                const float e = jd == 0 ? acc[m][0] : (jd == 1 ? acc[m][1] : (jd == 2 ? acc[m][2] : acc[m][3]));
                if (I == J && jd >= 0 && jd < 4 && 16 * I + q16 < A.bw) dm = fmaxf(dm, e);
            }
#pragma unroll
            for (int s2 = 1; s2 < 64; s2 <<= 1) dm = fmaxf(dm, __shfl_xor(dm, s2));
            if (lane == 0) lds_big[L::DM + I1] = dm;
        }
        __syncthreads();  // every wave is done with its staging before the tiles land on it
#pragma unroll
        for (int m = 0; m <= NT; ++m) {
            int I, J;
            tile_of(m, I1, NT, I, J);
            tile_store<TP>(mat + tile_id(I, J) * TSZ, acc[m], lane);
        }
        __syncthreads();

        // Blocked LDL^T on the tiles in LDS with the forward substitution folded in.  Wave 0
        // factors each 16-column panel with a lane per row (lane l holds rows l, 64 + l, ...);
        // every wave then applies the panel to its own tiles on the matrix cores.
        float* zero = lds_big + L::YP;  // 16 x 16 zeros at pitch TP (back substitution)
        float* pvl = zero + TSZ;        // [B] pivots
#pragma unroll 1
        for (int K = 0; K < NT; ++K) {
            big_panel<NT>(mat, pvl, gl, lane, I1, K);
            __syncthreads();
            // trailing tiles: A_IJ -= L_IK diag(piv) L_JK^T for K < J <= I (the panel holds -L)
#pragma unroll 1
            for (int pass = 0; pass < 2; ++pass) {
                const int I = pass == 0 ? I1 : I2;
                if (I <= K) continue;
                const float* LI = mat + tile_id(I, K) * TSZ;
#pragma unroll 1
                for (int J = K + 1; J <= I; ++J) {
                    float* T = mat + tile_id(I, J) * TSZ;
                    floatx4 c = tile_load<TP>(T, lane);
                    c = mm_pdqt<TP>(c, LI, mat + tile_id(J, K) * TSZ, pvl + 16 * K, lane);
                    tile_store<TP>(T, c, lane);
                }
            }
            __syncthreads();
        }
        // pivot check over the real coordinates (every wave, from LDS)
        // against the largest diagonal entry of the Hessian: the pivots lie between the smallest
        // eigenvalue and the diagonal entries, so the ratio bounds the condition number from below
        float pmin = 3.0e38f, dmax = 0.f;
        bool nonpos_l = false;  // NaN pivots too (fminf skips NaNs)
#pragma unroll
        for (int h = 0; h < NH; ++h) {
            const int q = 64 * h + lane;
            const float v = pvl[q];
            if (q < A.bw) {
                pmin = fminf(pmin, v);
                nonpos_l = nonpos_l || !(v > 0.f);
            }
        }
#pragma unroll
        for (int w = 0; w < L::NW; ++w) dmax = fmaxf(dmax, lds_big[L::DM + w]);
        const bool nonpos = __ballot(nonpos_l) != 0;
#pragma unroll
        for (int m = 1; m < 64; m <<= 1) pmin = fminf(pmin, __shfl_xor(pmin, m));
        const int bad = __builtin_amdgcn_readfirstlane((nonpos || !(pmin > 0.f) || (pmin < A.tau * dmax)) ? 1 : 0);
        if (bad) {
            if (lead && lane == 0) {
                const int pos = atomicAdd(&A.cursors[CUR_FB_LIST], 1);
                A.fb_list[pos] = r;
            }
            __syncthreads();
            continue;
        }
        if (I1 == 0) {
            // w = D^-1 L^-1 g, then L^T x = w from the last column (see the narrow kernel)
            float w[NH];
#pragma unroll
            for (int h = 0; h < NH; ++h) w[h] = gl[64 * h + lane] * __builtin_amdgcn_rcpf(pvl[64 * h + lane]);
#pragma unroll 1
            for (int K = NT - 1; K >= 0; --K) {
                const float* rowp[NH];
#pragma unroll
                for (int h = 0; h < NH; ++h) {
                    const int ti = 4 * h + (lane >> 4);  // tile column of this lane's row
                    rowp[h] = (ti <= K) ? mat + tile_id(K, ti) * TSZ + (lane & 15) : zero + (lane & 15);
                }
                float lt[NH][16];
#pragma unroll
                for (int h = 0; h < NH; ++h)
#pragma unroll
                    for (int jj = 0; jj < 16; ++jj) lt[h][jj] = rowp[h][jj * TP];
                const int hk = K >> 2;
                float wk = w[0];
#pragma unroll
                for (int h = 1; h < NH; ++h) wk = (hk == h) ? w[h] : wk;
#pragma unroll
                for (int jj = 15; jj >= 0; --jj) {
                    const float xk = readlane(wk, 16 * (K & 3) + jj);
#pragma unroll
                    for (int h = 0; h < NH; ++h) w[h] = fmaf(lt[h][jj], xk, w[h]);
                    wk = w[0];
#pragma unroll
                    for (int h = 1; h < NH; ++h) wk = (hk == h) ? w[h] : wk;
                }
            }
#pragma unroll
            for (int h = 0; h < NH; ++h) {
                const int q = 64 * h + lane;
                if (q < A.bw) A.X[(size_t)r * A.d + A.p0 + q] -= w[h];
            }
        }
        __syncthreads();
    }
}

// Float64 redo of rejected rows for wide blocks: the Hessian lives in a global float64
// scratch (one B x B per workgroup), gathered rows come through LDS in chunks of 8.
template <int NT>
__global__ __launch_bounds__(256) void k_fallback_big(SweepArgs A) {
    constexpr int B = 16 * NT, CH = 8;
    __shared__ double xs[CH][B];
    __shared__ double gv[B], own[B];
    __shared__ double rs[CH], ws[CH];
    __shared__ int ok;
    const int tid = threadIdx.x;
    double* Hm = A.fb_scratch + (size_t)blockIdx.x * B * B;
    const int nfb = A.cursors[CUR_FB_LIST];
    for (int idx = blockIdx.x; idx < nfb; idx += gridDim.x) {
        const int r = A.fb_list[idx];
        const int64_t lo = A.ptr[r], hi = A.ptr[r + 1];
        for (int e = tid; e < B * B; e += 256) Hm[e] = (double)A.Dmat[e];
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
                Hm[e] += s;
            }
            if (tid < B) {
                double s = 0.0;
                for (int j = 0; j < CH; ++j) s += rs[j] * xs[j][tid];
                gv[tid] += s;
            }
            __syncthreads();
        }
        // right-looking Cholesky in float64 (lower triangle), the workgroup sharing each column
        for (int k = 0; k < B; ++k) {
            if (tid == 0) {
                double v = Hm[(size_t)k * B + k];
                if (!(v > 0.0)) {
                    ok = 0;
                    v = 1.0;
                }
                Hm[(size_t)k * B + k] = sqrt(v);
            }
            __syncthreads();
            for (int i = k + 1 + tid; i < B; i += 256) Hm[(size_t)i * B + k] /= Hm[(size_t)k * B + k];
            __syncthreads();
            const int t = B - k - 1;
            for (int e = tid; e < t * t; e += 256) {
                const int i = k + 1 + e / t, j = k + 1 + e % t;
                if (j <= i) Hm[(size_t)i * B + j] -= Hm[(size_t)i * B + k] * Hm[(size_t)j * B + k];
            }
            __syncthreads();
        }
        if (tid == 0) {
            for (int i = 0; i < B; ++i) {
                double s = gv[i];
                for (int k = 0; k < i; ++k) s -= Hm[(size_t)i * B + k] * gv[k];
                gv[i] = s / Hm[(size_t)i * B + i];
            }
            for (int i = B - 1; i >= 0; --i) {
                double s = gv[i];
                for (int k = i + 1; k < B; ++k) s -= Hm[(size_t)k * B + i] * gv[k];
                gv[i] = s / Hm[(size_t)i * B + i];
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

constexpr int kFallbackBlocksBig = 64;

template <int NT, bool TRANS, bool BF>
void launch_big_nt(ials_ctx* c, const SweepArgs& args, const SideIndex& s, int sd) {
    using L = BigLds<NT>;
    hipStream_t st = c->stream;
    const unsigned threads = NT * 32;
    if (s.nseg > 0) {
        ProfScope ps(c, IALS_K_SEG_USER + sd);
        hipLaunchKernelGGL((k_seg_big<NT, TRANS, BF>), dim3(std::min<unsigned>((unsigned)c->num_cu * 4, (unsigned)s.nseg)),
                           dim3(threads), 0, st, args);
        launch_seg_group(st, args, big_seg_stride<NT>());
    }
    if (s.nrows > 0) {
        const size_t lds = sizeof(float) * L::TOTAL;
        static OccCache occ;
        const int resident = resident_per_cu(occ, reinterpret_cast<const void*>(&k_rows_big<NT, TRANS, BF>),
                                             (int)threads, lds, true, 1);
        {
            ProfScope ps(c, (TRANS ? IALS_K_ROWS_USER_MOVE : IALS_K_ROWS_USER) + sd);
            hipLaunchKernelGGL((k_rows_big<NT, TRANS, BF>),
                               dim3(std::min<unsigned>((unsigned)(c->num_cu * resident), (unsigned)s.nrows)),
                               dim3(threads), lds, st, args);
        }
        ProfScope ps(c, IALS_K_FALLBACK_USER + sd);
        hipLaunchKernelGGL((k_fallback_big<NT>), dim3(kFallbackBlocksBig), dim3(256), 0, st, args);
    }
}

template <int NT, bool BF>
void launch_big_b(ials_ctx* c, SweepArgs& A, const SideIndex& s, int sd, bool trans) {
    if (trans)
        launch_big_nt<NT, true, BF>(c, A, s, sd);
    else
        launch_big_nt<NT, false, BF>(c, A, s, sd);
}

}  // namespace

size_t big_fallback_doubles(int32_t B) { return (size_t)kFallbackBlocksBig * B * B; }

void launch_fallback_big(ials_ctx* c, const SweepArgs& A) {
    if (c->B == 128)
        hipLaunchKernelGGL((k_fallback_big<8>), dim3(kFallbackBlocksBig), dim3(256), 0, c->stream, A);
    else
        hipLaunchKernelGGL((k_fallback_big<16>), dim3(kFallbackBlocksBig), dim3(256), 0, c->stream, A);
}

void launch_sweep_big(ials_ctx* c, SweepArgs& A, const SideIndex& s, int sd, bool trans) {
    const bool bf = c->precision == IALS_PREC_BF16;
    A.fb_scratch = c->fb_scratch;
    if (c->B == 128) {
        if (bf)
            launch_big_b<8, true>(c, A, s, sd, trans);
        else
            launch_big_b<8, false>(c, A, s, sd, trans);
    } else {
        if (bf)
            launch_big_b<16, true>(c, A, s, sd, trans);
        else
            launch_big_b<16, false>(c, A, s, sd, trans);
    }
}

}  // namespace ials
