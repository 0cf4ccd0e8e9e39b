// Dense kernels of an iALS++ pass (gfx950, wave64):
//   k_predict     yhat = <w_u, h_i> for every observation (eq. 1; first step of an epoch, Alg. 3)
//   k_gram_part   partial Gramian X^T X[:, pi] (eq. 7), split over row chunks, MFMA f32 16x16x4
//   k_gram_reduce fixed-order float64 sum of the chunk partials
//   k_make_dmat   alpha0 * G_{pi,pi} + lambda I (the Hessian's dense part, eq. 9)
//   k_dense       alpha0 * x_r G^{pi} + lambda x_{r,pi} for every row (the gradient's dense part, eq. 8)
//   loss kernels  eq. 2 in float64: observed term from fresh predictions and
//                 <W^T W, H^T H>_F with both Gramians formed in float64.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "ials_internal.h"

namespace ials {
namespace {

__device__ inline floatx4 mfma4(float a, float b, floatx4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

inline unsigned nblk(int64_t n, int t) { return (unsigned)((n + t - 1) / t); }

// Prediction cache relative to a block pi = [p0, p0+bw) (eq. 1 split in two parts):
//   inside == false:  out_k = sum over f outside pi of w_u[f] h_i[f]
//   inside == true:   out_k = base_k + sum over f inside pi of w_u[f] h_i[f]
// With inside == false this is the cache a pass of block pi starts from
// (yhat = out + <w_{u,pi}, h_{i,pi}>); with inside == true it turns the cache back
// into yhat.  One wavefront per user; 16 lanes per observation, 4 at a time.
__global__ __launch_bounds__(256) void k_predict(int32_t U, int32_t d, const int64_t* __restrict__ ptr,
                                                 const int32_t* __restrict__ col, const float* __restrict__ W,
                                                 const float* __restrict__ H, int32_t p0, int32_t bw, bool inside,
                                                 const float* __restrict__ base, float* __restrict__ out) {
    const int u = (int)((blockIdx.x * 256u + threadIdx.x) >> 6);
    const int lane = threadIdx.x & 63, q16 = lane & 15, g4 = lane >> 4;
    if (u >= U) return;
    const float* w = W + (size_t)u * d;
    const int64_t lo = ptr[u], hi = ptr[u + 1];
    for (int64_t k0 = lo; k0 < hi; k0 += 4) {
        const int64_t k = k0 + g4;
        const bool v = k < hi;
        const float* h = H + (size_t)(v ? col[k] : 0) * d;
        float s = 0.f;
        for (int f = q16; f < d; f += 16) {
            const bool in = f >= p0 && f < p0 + bw;
            if (in == inside) s = fmaf(w[f], h[f], s);
        }
        s = row_sum16(s);
        if (v && q16 == 0) out[k] = inside ? base[k] + s : s;
    }
}

// Same computation for d = 64*J with the row held in registers: only the JL chunks of 64
// columns listed in ch take part (chunks wholly inside, or wholly outside, the summed
// range are skipped, so the partner rows are read only where they count; within a listed
// chunk the excluded or included columns are masked once per row).  The partner ids of 64
// observations are loaded at once and 8 observations' rows are in flight per 16-lane group.
template <int J, int JL>
__global__ __launch_bounds__(256) void k_predict_rows(int32_t U, const int64_t* __restrict__ ptr,
                                                      const int32_t* __restrict__ col, const float* __restrict__ W,
                                                      const float* __restrict__ H, int32_t p0, int32_t bw, bool inside,
                                                      int4 ch, const float* __restrict__ base, float* __restrict__ out) {
    constexpr int D = 64 * J;
    const int u = (int)((blockIdx.x * 256u + threadIdx.x) >> 6);
    const int lane = threadIdx.x & 63, q16 = lane & 15, g4 = lane >> 4;
    if (u >= U) return;
    const int chs[4] = {ch.x, ch.y, ch.z, ch.w};
    float4 w[JL];
#pragma unroll
    for (int j = 0; j < JL; ++j) {
        const int f = 4 * q16 + 64 * chs[j];
        float4 v = *reinterpret_cast<const float4*>(W + (size_t)u * D + f);
        v.x = ((f + 0 >= p0 && f + 0 < p0 + bw) == inside) ? v.x : 0.f;
        v.y = ((f + 1 >= p0 && f + 1 < p0 + bw) == inside) ? v.y : 0.f;
        v.z = ((f + 2 >= p0 && f + 2 < p0 + bw) == inside) ? v.z : 0.f;
        v.w = ((f + 3 >= p0 && f + 3 < p0 + bw) == inside) ? v.w : 0.f;
        w[j] = v;
    }
    const int64_t lo = ptr[u], hi = ptr[u + 1];
    for (int64_t c0 = lo; c0 < hi; c0 += 64) {
        const int64_t k = c0 + lane;
        const int ci = (k < hi) ? col[k] : 0;
        const int cnt = (int)min((int64_t)64, hi - c0);
        const int nsteps = (cnt + 3) >> 2;
        for (int st = 0; st < nsteps; st += 8) {
            // eight steps' rows loaded together (steps past the chunk read a valid row, unused)
            float4 h[8][JL];
#pragma unroll
            for (int v = 0; v < 8; ++v) {
                const int i = __shfl(ci, (4 * (st + v) + g4) & 63);
#pragma unroll
                for (int j = 0; j < JL; ++j)
                    h[v][j] = *reinterpret_cast<const float4*>(H + (size_t)i * D + 4 * q16 + 64 * chs[j]);
            }
#pragma unroll
            for (int v = 0; v < 8; ++v) {
                float s = 0.f;
#pragma unroll
                for (int j = 0; j < JL; ++j) {
                    s = fmaf(w[j].x, h[v][j].x, s);
                    s = fmaf(w[j].y, h[v][j].y, s);
                    s = fmaf(w[j].z, h[v][j].z, s);
                    s = fmaf(w[j].w, h[v][j].w, s);
                }
                s = row_sum16(s);
                const int idx = 4 * (st + v) + g4;
                if (q16 == 0 && idx < cnt) out[c0 + idx] = inside ? base[c0 + idx] + s : s;
            }
        }
    }
}

// The same for d = 256 J (J >= 2) with the whole wavefront on one observation: lane l
// holds w_u[f] for f = 4 l + 256 j (j < J) and loads the same columns of h_i, UB observations
// at a time with all their loads in flight, then each dot product is summed over the wave.
__device__ inline float readlane_f(float x, int l) {
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x), l));
}
template <int J, int UB>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(1, 4))) void k_predict_wide(int32_t U, const int64_t* __restrict__ ptr,
                                                      const int32_t* __restrict__ col, const float* __restrict__ W,
                                                      const float* __restrict__ H, int32_t p0, int32_t bw, bool inside,
                                                      const float* __restrict__ base, float* __restrict__ out) {
    constexpr int D = 256 * J;
    const int u = (int)((blockIdx.x * 256u + threadIdx.x) >> 6);
    const int lane = threadIdx.x & 63;
    if (u >= U) return;
    float4 w[J];
#pragma unroll
    for (int j = 0; j < J; ++j) {
        float4 v = *reinterpret_cast<const float4*>(W + (size_t)u * D + 4 * lane + 256 * j);
        const int f = 4 * lane + 256 * j;
        v.x = ((f + 0 >= p0 && f + 0 < p0 + bw) == inside) ? v.x : 0.f;
        v.y = ((f + 1 >= p0 && f + 1 < p0 + bw) == inside) ? v.y : 0.f;
        v.z = ((f + 2 >= p0 && f + 2 < p0 + bw) == inside) ? v.z : 0.f;
        v.w = ((f + 3 >= p0 && f + 3 < p0 + bw) == inside) ? v.w : 0.f;
        w[j] = v;
    }
    const int64_t lo = ptr[u], hi = ptr[u + 1];
    for (int64_t c0 = lo; c0 < hi; c0 += 64) {
        const int64_t k = c0 + lane;
        const int ci = (k < hi) ? col[k] : 0;
        const int cnt = (int)min((int64_t)64, hi - c0);
        float mine = 0.f;  // lane t keeps the prediction of observation c0 + t
        for (int t0 = 0; t0 < cnt; t0 += UB) {
            float4 h[UB][J];
#pragma unroll
            for (int v = 0; v < UB; ++v) {
                const int i = __shfl(ci, (t0 + v) & 63);  // past the chunk: a valid row, result unused
#pragma unroll
                for (int j = 0; j < J; ++j)
                    h[v][j] = *reinterpret_cast<const float4*>(H + (size_t)i * D + 4 * lane + 256 * j);
            }
#pragma unroll
            for (int v = 0; v < UB; ++v) {
                float s = 0.f;
#pragma unroll
                for (int j = 0; j < J; ++j) {
                    s = fmaf(w[j].x, h[v][j].x, s);
                    s = fmaf(w[j].y, h[v][j].y, s);
                    s = fmaf(w[j].z, h[v][j].z, s);
                    s = fmaf(w[j].w, h[v][j].w, s);
                }
                // the 64-lane sum: each 16-lane row summed by DPP rotations, the four row
                // sums read as scalars
                s = row_sum16(s);
                const float tot = (readlane_f(s, 0) + readlane_f(s, 16)) + (readlane_f(s, 32) + readlane_f(s, 48));
                if (lane == t0 + v) mine = tot;
            }
        }
        if (lane < cnt) out[c0 + lane] = inside ? base[c0 + lane] + mine : mine;
    }
}

// The same over the columns [f0, f0 + 256 J) of rows of d columns: the first slice writes
// its partial dot products (on top of base with inside), the later ones add theirs.  Slices
// whose rows of H fit the Infinity Cache (256 MB) are re-read from it instead of HBM: the
// observations of a user visit random items, each item row about |S| / |I| times per pass.
template <int J, int UB>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(1, 4))) void k_predict_slice(
    int32_t U, int32_t d, int32_t f0, bool first, const int64_t* __restrict__ ptr, const int32_t* __restrict__ col,
    const float* __restrict__ W, const float* __restrict__ H, int32_t p0, int32_t bw, bool inside,
    const float* __restrict__ base, float* __restrict__ out) {
    const int u = (int)((blockIdx.x * 256u + threadIdx.x) >> 6);
    const int lane = threadIdx.x & 63;
    if (u >= U) return;
    float4 w[J];
#pragma unroll
    for (int j = 0; j < J; ++j) {
        const int f = f0 + 4 * lane + 256 * j;
        // each row of W is read once per pass: streamed past the caches
        const floatx4 nv = __builtin_nontemporal_load(reinterpret_cast<const floatx4*>(W + (size_t)u * d + f));
        float4 v = make_float4(nv[0], nv[1], nv[2], nv[3]);
        v.x = ((f + 0 >= p0 && f + 0 < p0 + bw) == inside) ? v.x : 0.f;
        v.y = ((f + 1 >= p0 && f + 1 < p0 + bw) == inside) ? v.y : 0.f;
        v.z = ((f + 2 >= p0 && f + 2 < p0 + bw) == inside) ? v.z : 0.f;
        v.w = ((f + 3 >= p0 && f + 3 < p0 + bw) == inside) ? v.w : 0.f;
        w[j] = v;
    }
    const int64_t lo = ptr[u], hi = ptr[u + 1];
    for (int64_t c0 = lo; c0 < hi; c0 += 64) {
        const int64_t k = c0 + lane;
        const int ci = (k < hi) ? col[k] : 0;
        const int cnt = (int)min((int64_t)64, hi - c0);
        float mine = 0.f;  // lane t keeps the partial prediction of observation c0 + t
        for (int t0 = 0; t0 < cnt; t0 += UB) {
            float4 h[UB][J];
#pragma unroll
            for (int v = 0; v < UB; ++v) {
                const int i = __shfl(ci, (t0 + v) & 63);  // past the chunk: a valid row, result unused
#pragma unroll
                for (int j = 0; j < J; ++j)
                    h[v][j] = *reinterpret_cast<const float4*>(H + (size_t)i * d + f0 + 4 * lane + 256 * j);
            }
#pragma unroll
            for (int v = 0; v < UB; ++v) {
                float s = 0.f;
#pragma unroll
                for (int j = 0; j < J; ++j) {
                    s = fmaf(w[j].x, h[v][j].x, s);
                    s = fmaf(w[j].y, h[v][j].y, s);
                    s = fmaf(w[j].z, h[v][j].z, s);
                    s = fmaf(w[j].w, h[v][j].w, s);
                }
                // the 64-lane sum: each 16-lane row summed by DPP rotations, the four row
                // sums read as scalars
                s = row_sum16(s);
                const float tot = (readlane_f(s, 0) + readlane_f(s, 16)) + (readlane_f(s, 32) + readlane_f(s, 48));
                if (lane == t0 + v) mine = tot;
            }
        }
        if (lane < cnt) {
            const float prev = first ? (inside ? base[c0 + lane] : 0.f) : out[c0 + lane];
            out[c0 + lane] = prev + mine;
        }
    }
}

// Partial Gramian of one row chunk: part[chunk][f][q] = sum_{r in chunk} X[r][f] X[r][p0+q]
// for f < d, q < ncols (columns q >= bw are zero).  Block = one wavefront owning a
// 64 x (16*QT) output tile (4 x QT MFMA tiles).  BF: bfloat16 operands (16 rows per
// 16x16x16 MFMA, four rows per lane), float32 accumulation.
__device__ inline unsigned bf16_bits(float f) {
    const unsigned u = __float_as_uint(f);
    return (u + 0x7fffu + ((u >> 16) & 1u)) >> 16;
}
__device__ inline shortx4 bf16x4(const float* v) {
    return shortx4{(short)bf16_bits(v[0]), (short)bf16_bits(v[1]), (short)bf16_bits(v[2]), (short)bf16_bits(v[3])};
}

template <int QT, bool BF>
__global__ __launch_bounds__(64) void k_gram_part(int32_t n, int32_t d, const float* __restrict__ X, int32_t p0,
                                                  int32_t bw, int32_t ncols, int32_t rows_per_chunk,
                                                  float* __restrict__ part) {
    const int lane = threadIdx.x, q16 = lane & 15, g4 = lane >> 4;
    const int f0 = blockIdx.x * 64, qg0 = blockIdx.y * 16 * QT;
    const int chunk = blockIdx.z;
    const int64_t r0 = (int64_t)chunk * rows_per_chunk;
    const int64_t r1 = std::min<int64_t>(n, r0 + rows_per_chunk);
    floatx4 acc[4][QT];
#pragma unroll
    for (int ft = 0; ft < 4; ++ft)
#pragma unroll
        for (int qt = 0; qt < QT; ++qt) acc[ft][qt] = floatx4{0.f, 0.f, 0.f, 0.f};
    if constexpr (BF) {
        for (int64_t r = r0; r < r1; r += 16) {
            float a[4][4], b[QT][4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int64_t rr = r + 4 * g4 + u;
                const bool v = rr < r1;
                const float* xr = X + (size_t)(v ? rr : 0) * d;
#pragma unroll
                for (int ft = 0; ft < 4; ++ft) {
                    const int f = f0 + 16 * ft + q16;
                    a[ft][u] = (v && f < d) ? xr[f] : 0.f;
                }
#pragma unroll
                for (int qt = 0; qt < QT; ++qt) {
                    const int q = qg0 + 16 * qt + q16;
                    b[qt][u] = (v && q < bw) ? xr[p0 + q] : 0.f;
                }
            }
            shortx4 pa[4], pb[QT];
#pragma unroll
            for (int ft = 0; ft < 4; ++ft) pa[ft] = bf16x4(a[ft]);
#pragma unroll
            for (int qt = 0; qt < QT; ++qt) pb[qt] = bf16x4(b[qt]);
#pragma unroll
            for (int ft = 0; ft < 4; ++ft)
#pragma unroll
                for (int qt = 0; qt < QT; ++qt)
                    acc[ft][qt] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(pa[ft], pb[qt], acc[ft][qt], 0, 0, 0);
        }
    } else {
        for (int64_t r = r0; r < r1; r += 4) {
            const int64_t rr = r + g4;
            const bool v = rr < r1;
            const float* xr = X + (size_t)(v ? rr : 0) * d;
            float a[4], b[QT];
#pragma unroll
            for (int ft = 0; ft < 4; ++ft) {
                const int f = f0 + 16 * ft + q16;
                a[ft] = (v && f < d) ? xr[f] : 0.f;
            }
#pragma unroll
            for (int qt = 0; qt < QT; ++qt) {
                const int q = qg0 + 16 * qt + q16;
                b[qt] = (v && q < bw) ? xr[p0 + q] : 0.f;
            }
#pragma unroll
            for (int ft = 0; ft < 4; ++ft)
#pragma unroll
                for (int qt = 0; qt < QT; ++qt) acc[ft][qt] = mfma4(a[ft], b[qt], acc[ft][qt]);
        }
    }
    float* out = part + (size_t)chunk * d * ncols;
#pragma unroll
    for (int ft = 0; ft < 4; ++ft)
#pragma unroll
        for (int qt = 0; qt < QT; ++qt)
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int f = f0 + 16 * ft + 4 * g4 + j, q = qg0 + 16 * qt + q16;
                if (f < d && q < ncols) out[(size_t)f * ncols + q] = acc[ft][qt][j];
            }
}

// The same partial on full 64 x 64 tiles with 16-byte loads, for d a multiple of 64 and a
// block of a multiple of 64 columns fully inside the row: lane q16 loads columns
// 4 q16 .. 4 q16 + 3 of a row, so MFMA tile j holds the columns congruent to j mod 4 (row m
// of tile ft is f = f0 + 4 m + ft, column n of tile qt is q = q0 + 4 n + qt).  The four
// wavefronts of a block take interleaved groups of 16 rows of the chunk; their partials are
// added in LDS in wavefront order, so one partial per block is written.
// Two operand sets alternate: the rows of the next group are loaded while the current group
// is multiplied.  The loads have no branches (rows past the chunk read its first row and
// their weight z is 0), and the sets are never copied, so waiting for the current operands
// does not wait for the ones in flight.
// k_gram_vec with the rows read by buffer loads over the chunk: the descriptor's range ends at
// the chunk's last row, so rows past it read as zeros (no masking), and every load takes its row
// offset from one uniform register and its column offset from a per-lane constant (no address
// arithmetic in the loop).  Needs (rows_per_chunk + 160) * d * 4 < 2^31.
__global__ __launch_bounds__(256, 2) void k_gram_buf(int32_t n, int32_t d, const float* __restrict__ X, int32_t p0,
                                                  int32_t ncols, int32_t rows_per_chunk, float* __restrict__ part) {
    __shared__ floatx4 red[3][16][64];
    // the wavefront index is uniform; saying so keeps the row offset of the loads in a scalar register
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63, q16 = lane & 15,
              g4 = lane >> 4;
    const int f0 = blockIdx.x * 64, q0 = blockIdx.y * 64;
    const int64_t r0 = (int64_t)blockIdx.z * rows_per_chunk;
    const int64_t r1 = std::min<int64_t>(n, r0 + rows_per_chunk);
    floatx4 acc[4][4];
#pragma unroll
    for (int ft = 0; ft < 4; ++ft)
#pragma unroll
        for (int qt = 0; qt < 4; ++qt) acc[ft][qt] = floatx4{0.f, 0.f, 0.f, 0.f};
    const int nbytes = (int)std::max<int64_t>(0, (r1 - r0) * d * 4);
    const __amdgpu_buffer_rsrc_t rs =
        __builtin_amdgcn_make_buffer_rsrc(const_cast<float*>(X + (size_t)r0 * d), (short)0, nbytes, 0x00020000);
    int oa[4], ob[4];
#pragma unroll
    for (int s = 0; s < 4; ++s) {
        oa[s] = ((4 * s + g4) * d + f0 + 4 * q16) * 4;
        ob[s] = ((4 * s + g4) * d + p0 + q0 + 4 * q16) * 4;
    }
    floatx4 a0[4], b0[4], a1[4], b1[4];
    auto load = [&](int rel, floatx4* a, floatx4* b) {
        const int so = rel * d * 4;
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            a[s] = __builtin_bit_cast(floatx4, __builtin_amdgcn_raw_buffer_load_b128(rs, oa[s], so, 0));
            b[s] = __builtin_bit_cast(floatx4, __builtin_amdgcn_raw_buffer_load_b128(rs, ob[s], so, 0));
        }
        __builtin_amdgcn_sched_barrier(0);  // keep the loads ahead of the next MFMA block
    };
    auto mma = [&](const floatx4* a, const floatx4* b) {
#pragma unroll
        for (int s = 0; s < 4; ++s)
#pragma unroll
            for (int ft = 0; ft < 4; ++ft)
#pragma unroll
                for (int qt = 0; qt < 4; ++qt) acc[ft][qt] = mfma4(a[s][ft], b[s][qt], acc[ft][qt]);
    };
    const int rows = (int)(r1 - r0);
    int rel = 16 * wave;
    load(rel, a0, b0);
    for (; rel < rows; rel += 128) {
        load(rel + 64, a1, b1);
        mma(a0, b0);
        load(rel + 128, a0, b0);
        mma(a1, b1);
    }
    if (wave > 0) {
#pragma unroll
        for (int ft = 0; ft < 4; ++ft)
#pragma unroll
            for (int qt = 0; qt < 4; ++qt) red[wave - 1][4 * ft + qt][lane] = acc[ft][qt];
    }
    __syncthreads();
    if (wave != 0) return;
#pragma unroll
    for (int w = 0; w < 3; ++w)
#pragma unroll
        for (int ft = 0; ft < 4; ++ft)
#pragma unroll
            for (int qt = 0; qt < 4; ++qt) acc[ft][qt] += red[w][4 * ft + qt][lane];
    float* out = part + (size_t)blockIdx.z * d * ncols + q0 + 4 * q16;
#pragma unroll
    for (int ft = 0; ft < 4; ++ft)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int f = f0 + 4 * (4 * g4 + j) + ft;
            *reinterpret_cast<float4*>(out + (size_t)f * ncols) =
                make_float4(acc[ft][0][j], acc[ft][1][j], acc[ft][2][j], acc[ft][3][j]);
        }
}

__global__ __launch_bounds__(256, 2) void k_gram_vec(int32_t n, int32_t d, const float* __restrict__ X, int32_t p0,
                                                  int32_t ncols, int32_t rows_per_chunk, float* __restrict__ part) {
    __shared__ floatx4 red[3][16][64];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, q16 = lane & 15, g4 = lane >> 4;
    const int f0 = blockIdx.x * 64, q0 = blockIdx.y * 64;
    const int64_t r0 = (int64_t)blockIdx.z * rows_per_chunk;
    const int64_t r1 = std::min<int64_t>(n, r0 + rows_per_chunk);
    floatx4 acc[4][4];
#pragma unroll
    for (int ft = 0; ft < 4; ++ft)
#pragma unroll
        for (int qt = 0; qt < 4; ++qt) acc[ft][qt] = floatx4{0.f, 0.f, 0.f, 0.f};
    const float* xa = X + f0 + 4 * q16;
    const float* xb = X + p0 + q0 + 4 * q16;
    floatx4 a0[4], b0[4], a1[4], b1[4];
    float z0[4], z1[4];
    auto load = [&](int64_t rb, floatx4* a, floatx4* b, float* z) {
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            const int64_t r = rb + 4 * s + g4;
            const bool in = r < r1;
            const int64_t rr = in ? r : r0;
            a[s] = *reinterpret_cast<const floatx4*>(xa + (size_t)rr * d);
            b[s] = *reinterpret_cast<const floatx4*>(xb + (size_t)rr * d);
            z[s] = in ? 1.f : 0.f;
        }
        __builtin_amdgcn_sched_barrier(0);  // keep the loads ahead of the next MFMA block
    };
    auto mma = [&](floatx4* a, const floatx4* b, const float* z) {
#pragma unroll
        for (int s = 0; s < 4; ++s) a[s] *= z[s];
#pragma unroll
        for (int s = 0; s < 4; ++s)
#pragma unroll
            for (int ft = 0; ft < 4; ++ft)
#pragma unroll
                for (int qt = 0; qt < 4; ++qt) acc[ft][qt] = mfma4(a[s][ft], b[s][qt], acc[ft][qt]);
    };
    int64_t rb = r0 + 16 * wave;
    load(rb, a0, b0, z0);
    for (; rb < r1; rb += 128) {
        load(rb + 64, a1, b1, z1);
        mma(a0, b0, z0);
        load(rb + 128, a0, b0, z0);
        mma(a1, b1, z1);
    }
    if (wave > 0) {
#pragma unroll
        for (int ft = 0; ft < 4; ++ft)
#pragma unroll
            for (int qt = 0; qt < 4; ++qt) red[wave - 1][4 * ft + qt][lane] = acc[ft][qt];
    }
    __syncthreads();
    if (wave != 0) return;
#pragma unroll
    for (int w = 0; w < 3; ++w)
#pragma unroll
        for (int ft = 0; ft < 4; ++ft)
#pragma unroll
            for (int qt = 0; qt < 4; ++qt) acc[ft][qt] += red[w][4 * ft + qt][lane];
    float* out = part + (size_t)blockIdx.z * d * ncols + q0 + 4 * q16;
#pragma unroll
    for (int ft = 0; ft < 4; ++ft)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int f = f0 + 4 * (4 * g4 + j) + ft;
            *reinterpret_cast<float4*>(out + (size_t)f * ncols) =
                make_float4(acc[ft][0][j], acc[ft][1][j], acc[ft][2][j], acc[ft][3][j]);
        }
}

// The bfloat16 form of k_gram_vec (same tiles, column mapping and output): rows are taken 32
// at a time, lane group g4 holding rows 8 g4 .. 8 g4 + 7 of them, converted to bfloat16 (round
// to nearest even, v_cvt_pk_bf16_f32) and multiplied with v_mfma_f32_16x16x32_bf16 (float32
// accumulation): 16 matrix instructions per 32 rows instead of 128.  Two operand sets alternate
// as in k_gram_vec; rows past the chunk read its first row and are zeroed before conversion.
typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
__global__ __launch_bounds__(256, 2) void k_gram_vec_bf16(int32_t n, int32_t d, const float* __restrict__ X,
                                                       int32_t p0, int32_t ncols, int32_t rows_per_chunk,
                                                       float* __restrict__ part) {
    __shared__ floatx4 red[3][16][64];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, q16 = lane & 15, g4 = lane >> 4;
    const int f0 = blockIdx.x * 64, q0 = blockIdx.y * 64;
    const int64_t r0 = (int64_t)blockIdx.z * rows_per_chunk;
    const int64_t r1 = std::min<int64_t>(n, r0 + rows_per_chunk);
    floatx4 acc[4][4];
#pragma unroll
    for (int ft = 0; ft < 4; ++ft)
#pragma unroll
        for (int qt = 0; qt < 4; ++qt) acc[ft][qt] = floatx4{0.f, 0.f, 0.f, 0.f};
    const float* xa = X + f0 + 4 * q16;
    const float* xb = X + p0 + q0 + 4 * q16;
    floatx4 a0[8], b0[8], a1[8], b1[8];
    bool v0[8], v1[8];
    auto load = [&](int64_t rb, floatx4* a, floatx4* b, bool* v) {
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const int64_t r = rb + 8 * g4 + j;
            v[j] = r < r1;
            const int64_t rr = v[j] ? r : r0;
            a[j] = *reinterpret_cast<const floatx4*>(xa + (size_t)rr * d);
            b[j] = *reinterpret_cast<const floatx4*>(xb + (size_t)rr * d);
        }
        __builtin_amdgcn_sched_barrier(0);  // keep the loads ahead of the next MFMA block
    };
    auto mma = [&](const floatx4* a, const floatx4* b, const bool* v) {
        bf16x8_t pa[4], pb[4];
#pragma unroll
        for (int t = 0; t < 4; ++t)
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                pa[t][j] = (__bf16)(v[j] ? a[j][t] : 0.f);
                pb[t][j] = (__bf16)b[j][t];
            }
#pragma unroll
        for (int ft = 0; ft < 4; ++ft)
#pragma unroll
            for (int qt = 0; qt < 4; ++qt)
                acc[ft][qt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(pa[ft], pb[qt], acc[ft][qt], 0, 0, 0);
    };
    int64_t rb = r0 + 32 * wave;
    load(rb, a0, b0, v0);
    for (; rb < r1; rb += 256) {
        load(rb + 128, a1, b1, v1);
        mma(a0, b0, v0);
        load(rb + 256, a0, b0, v0);
        mma(a1, b1, v1);
    }
    if (wave > 0) {
#pragma unroll
        for (int ft = 0; ft < 4; ++ft)
#pragma unroll
            for (int qt = 0; qt < 4; ++qt) red[wave - 1][4 * ft + qt][lane] = acc[ft][qt];
    }
    __syncthreads();
    if (wave != 0) return;
#pragma unroll
    for (int w = 0; w < 3; ++w)
#pragma unroll
        for (int ft = 0; ft < 4; ++ft)
#pragma unroll
            for (int qt = 0; qt < 4; ++qt) acc[ft][qt] += red[w][4 * ft + qt][lane];
    float* out = part + (size_t)blockIdx.z * d * ncols + q0 + 4 * q16;
#pragma unroll
    for (int ft = 0; ft < 4; ++ft)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int f = f0 + 4 * (4 * g4 + j) + ft;
            *reinterpret_cast<float4*>(out + (size_t)f * ncols) =
                make_float4(acc[ft][0][j], acc[ft][1][j], acc[ft][2][j], acc[ft][3][j]);
        }
}

// ---- Full Gramian in bfloat16 (X^T X, d a multiple of 256): LDS-staged 256 x 256 tiles ----
//
// A workgroup of eight wavefronts forms one lower 256 x 256 tile (I >= J) of X^T X over one
// chunk of rows.  Per stage of 32 rows every thread loads an 8-row x 4-column block of the
// tile's two column strips (float32, 16-byte loads, the next stage's loads in flight while the
// current stage is multiplied), rounds it to bfloat16 (round to nearest even) and stores each
// column's 8 values as one 16-byte LDS write, so that LDS holds, per column, the stage's 32
// rows in order (a pitch of 40 bfloat16 spreads the 16-byte accesses over all banks).  Wavefront
// (wf, wq) multiplies columns 128 wf .. +127 of strip I by columns 64 wq .. +63 of strip J:
// 8 x 4 tiles of v_mfma_f32_16x16x32_bf16 per stage, each operand one 16-byte LDS read.  A
// diagonal tile reads both operands from strip I.  The 256-wide edge quarters the strip reads
// per product of the 64-wide tiles, which is what bounds the register-only kernel above.
// Workgroups of one chunk sit on the same XCD (blocks are dealt to XCDs round-robin), so the
// chunk's rows come from HBM once and from that XCD's L2 for the other tiles.
constexpr int kGLT = 256;                      // tile edge
constexpr int kGLK = 32;                       // rows per stage
constexpr int kGLP = 40;                       // LDS pitch of one column, in bfloat16
constexpr int kGLStrip = kGLT * kGLP;          // bfloat16 per strip
constexpr size_t kGLLds = 4 * kGLStrip * 2;    // two stages x two strips, in bytes
constexpr int kGLTileFloats = kGLT * kGLT;

int gram_lds_tiles(int32_t d) {
    const int T = d / kGLT;
    return T * (T + 1) / 2;
}
int gram_lds_chunks(int64_t n, int32_t d) {
    const int tiles = gram_lds_tiles(d);
    int64_t chunks = std::max(1, 256 / tiles);
    chunks = std::min<int64_t>(chunks, std::max<int64_t>(1, (n + kGLK - 1) / kGLK));
    return (int)chunks;
}

__global__ __launch_bounds__(512, 1) void k_gram_bf16_lds(int32_t n, int32_t d, const float* __restrict__ X,
                                                          int32_t tiles, int32_t chunks, int32_t per_xcd,
                                                          int32_t rows_per_chunk, float* __restrict__ part) {
    extern __shared__ __align__(16) __bf16 gl_lds[];
    // blocks b and b + 8 share an XCD: consecutive (chunk, tile) pairs go to the same XCD
    const int xcd = blockIdx.x & 7, slot = blockIdx.x >> 3;
    const int pair = xcd * per_xcd + slot;
    if (pair >= tiles * chunks) return;
    const int chunk = pair / tiles, tile = pair - chunk * tiles;
    int I = 0;
    while ((I + 1) * (I + 2) / 2 <= tile) ++I;
    const int J = tile - I * (I + 1) / 2;
    const bool diag = I == J;
    const int64_t r0 = (int64_t)chunk * rows_per_chunk;
    const int64_t r1 = std::min<int64_t>(n, r0 + rows_per_chunk);

    const int t = threadIdx.x, wave = t >> 6, lane = t & 63, q16 = lane & 15, g4 = lane >> 4;
    // loader role: strip s (0: columns of I, 1: columns of J), row group rg, column group cg
    const int s = t >> 8, rg = t & 3, cg = (t >> 2) & 63;
    const bool loader = !(diag && s == 1);
    // rows at or past r1 read as zeros: the buffer's range ends at row r1 (byte offsets are 32-bit,
    // the launcher checks that every row of X fits)
    const __amdgpu_buffer_rsrc_t rsrc =
        __builtin_amdgcn_make_buffer_rsrc(const_cast<float*>(X), (short)0, (int)(r1 * d * 4), 0x00020000);
    const uint32_t col_bytes = (uint32_t)((s == 0 ? I : J) * kGLT + 4 * cg) * 4;
    // the next stage's rows are loaded while the current stage is multiplied
    float4 va[8];
    auto load = [&](float4* v, int64_t k0) {
        if (!loader) return;
        const uint32_t o = (uint32_t)(k0 + 8 * rg) * (uint32_t)(4 * d) + col_bytes;
#pragma unroll
        for (int j = 0; j < 8; ++j)
            v[j] = __builtin_bit_cast(float4, __builtin_amdgcn_raw_buffer_load_b128(rsrc, o + (uint32_t)(j * 4 * d), 0, 0));
    };
    auto store = [&](const float4* v, int buf) {
        if (!loader) return;
        __bf16* base = gl_lds + (2 * buf + s) * kGLStrip + (4 * cg) * kGLP + 8 * rg;
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            bf16x8_t w;
#pragma unroll
            for (int j = 0; j < 8; ++j) w[j] = (__bf16)(c == 0 ? v[j].x : (c == 1 ? v[j].y : (c == 2 ? v[j].z : v[j].w)));
            *reinterpret_cast<bf16x8_t*>(base + c * kGLP) = w;
        }
    };

    const int wf = wave >> 2, wq = wave & 3;
    floatx4 acc[8][4];
#pragma unroll
    for (int ft = 0; ft < 8; ++ft)
#pragma unroll
        for (int qt = 0; qt < 4; ++qt) acc[ft][qt] = floatx4{0.f, 0.f, 0.f, 0.f};
    auto mma = [&](int buf) {
        const __bf16* A = gl_lds + (2 * buf) * kGLStrip + (128 * wf + q16) * kGLP + 8 * g4;
        const __bf16* B = gl_lds + (2 * buf + (diag ? 0 : 1)) * kGLStrip + (64 * wq + q16) * kGLP + 8 * g4;
        bf16x8_t b[4];
#pragma unroll
        for (int qt = 0; qt < 4; ++qt) b[qt] = *reinterpret_cast<const bf16x8_t*>(B + 16 * qt * kGLP);
#pragma unroll
        for (int ft = 0; ft < 8; ++ft) {
            const bf16x8_t a = *reinterpret_cast<const bf16x8_t*>(A + 16 * ft * kGLP);
#pragma unroll
            for (int qt = 0; qt < 4; ++qt)
                acc[ft][qt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b[qt], acc[ft][qt], 0, 0, 0);
        }
    };
    const int nst = (int)std::max<int64_t>(0, (r1 - r0 + kGLK - 1) / kGLK);
    auto k0_of = [&](int st) { return r0 + (int64_t)st * kGLK; };
    if (nst > 0) {
        load(va, k0_of(0));
        store(va, 0);
    }
    __syncthreads();
    for (int st = 0; st < nst; ++st) {
        if (st + 1 < nst) load(va, k0_of(st + 1));
        mma(st & 1);
        if (st + 1 < nst) store(va, (st + 1) & 1);
        __syncthreads();
    }
    // partials in the register layout: ((wave * 8 + ft) * 4 + qt) * 64 + lane, four floats each
    float* out = part + ((size_t)chunk * tiles + tile) * kGLTileFloats;
#pragma unroll
    for (int ft = 0; ft < 8; ++ft)
#pragma unroll
        for (int qt = 0; qt < 4; ++qt)
            *reinterpret_cast<floatx4*>(out + ((size_t)((wave * 8 + ft) * 4 + qt) * 64 + lane) * 4) = acc[ft][qt];
}

// G (d x d) from the partials of k_gram_bf16_lds: each element of a lower tile summed over the
// chunks in float64 in chunk order, written at (f, q) and mirrored to (q, f); in a diagonal tile
// only the elements on or below the diagonal are taken, so G is exactly symmetric.
__global__ __launch_bounds__(256) void k_gram_lds_reduce(const float* __restrict__ part, int32_t tiles, int32_t chunks,
                                                         int32_t d, float* __restrict__ G) {
    const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (e >= (int64_t)tiles * kGLTileFloats) return;
    const int tile = (int)(e / kGLTileFloats), o = (int)(e - (int64_t)tile * kGLTileFloats);
    int I = 0;
    while ((I + 1) * (I + 2) / 2 <= tile) ++I;
    const int J = tile - I * (I + 1) / 2;
    const int r = o & 3, lane = (o >> 2) & 63, qt = (o >> 8) & 3, ft = (o >> 10) & 7, w = o >> 13;
    const int f = kGLT * I + 128 * (w >> 2) + 16 * ft + 4 * (lane >> 4) + r;
    const int q = kGLT * J + 64 * (w & 3) + 16 * qt + (lane & 15);
    if (I == J && f < q) return;
    double sum = 0.0;
    for (int c = 0; c < chunks; ++c) sum += (double)part[((size_t)c * tiles + tile) * kGLTileFloats + o];
    const float g = (float)sum;
    G[(size_t)f * d + q] = g;
    G[(size_t)q * d + f] = g;
}

// out[e] = sum over chunks of part[c][e] in float64.  A block owns 16 outputs; its
// 16 thread rows each sum every 16th chunk, and the 16 partial sums of an
// output are then added in a fixed order.
__global__ __launch_bounds__(256) void k_gram_reduce(const float* __restrict__ part, int32_t nchunks, int64_t count,
                                                     float* __restrict__ out32) {
    __shared__ double red[16][17];
    const int o = threadIdx.x & 15, c = threadIdx.x >> 4;
    const int64_t e = (int64_t)blockIdx.x * 16 + o;
    double s = 0.0;
    if (e < count)
        for (int ch = c; ch < nchunks; ch += 16) s += (double)part[(size_t)ch * count + e];
    red[c][o] = s;
    __syncthreads();
    if (c == 0 && e < count) {
        double t = 0.0;
        for (int k = 0; k < 16; ++k) t += red[k][o];
        out32[e] = (float)t;
    }
}

// Dmat = alpha0 * G[p0:p0+bw, 0:bw] + lambda I, identity on the padding; also
// resets the work-queue cursors used by the sweep kernels of this pass.
__global__ void k_make_dmat(const float* __restrict__ G, int32_t B, int32_t p0, int32_t bw, float alpha0,
                            float lambda, float* __restrict__ Dmat, int32_t* __restrict__ cursors) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e < CUR_NUM) cursors[e] = 0;
    if (e >= B * B) return;
    const int p = e / B, q = e % B;
    float v;
    if (p < bw && q < bw)
        v = alpha0 * G[(size_t)(p0 + p) * B + q] + (p == q ? lambda : 0.f);
    else
        v = (p == q) ? 1.f : 0.f;
    Dmat[e] = v;
}

// R0[r][q] = alpha0 * sum_f X[r][f] G[f][q] + lambda * X[r][p0+q] (0 on padding columns).
// One wavefront per 64 rows (4 row tiles) x 16*NT columns (NT tiles) starting at column
// 16*NT*blockIdx.y; G and R0 have B columns.
template <int NT>
__global__ __launch_bounds__(256) void k_dense(int32_t n, int32_t d, int32_t B, const float* __restrict__ X,
                                               const float* __restrict__ G, int32_t p0, int32_t bw, float alpha0,
                                               float lambda, float* __restrict__ R0) {
    const int wave = (int)((blockIdx.x * 256u + threadIdx.x) >> 6);
    const int lane = threadIdx.x & 63, q16 = lane & 15, g4 = lane >> 4;
    const int qb = 16 * NT * blockIdx.y;
    const int64_t r0 = (int64_t)wave * 64;
    if (r0 >= n) return;
    floatx4 acc[4][NT];
#pragma unroll
    for (int rt = 0; rt < 4; ++rt)
#pragma unroll
        for (int t = 0; t < NT; ++t) acc[rt][t] = floatx4{0.f, 0.f, 0.f, 0.f};
    for (int f = 0; f < d; f += 4) {
        const int ff = f + g4;
        const bool fv = ff < d;
        float a[4], b[NT];
#pragma unroll
        for (int rt = 0; rt < 4; ++rt) {
            const int64_t r = r0 + 16 * rt + q16;
            a[rt] = (fv && r < n) ? X[(size_t)r * d + ff] : 0.f;
        }
#pragma unroll
        for (int t = 0; t < NT; ++t) b[t] = fv ? G[(size_t)ff * B + qb + 16 * t + q16] : 0.f;
#pragma unroll
        for (int rt = 0; rt < 4; ++rt)
#pragma unroll
            for (int t = 0; t < NT; ++t) acc[rt][t] = mfma4(a[rt], b[t], acc[rt][t]);
    }
#pragma unroll
    for (int rt = 0; rt < 4; ++rt)
#pragma unroll
        for (int t = 0; t < NT; ++t)
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int64_t r = r0 + 16 * rt + 4 * g4 + j;
                const int q = qb + 16 * t + q16;
                if (r < n)
                    R0[(size_t)r * B + q] =
                        (q < bw) ? fmaf(alpha0, acc[rt][t][j], lambda * X[(size_t)r * d + p0 + q]) : 0.f;
            }
}

// The same with 16-byte loads along f, for d a multiple of 16 and B a multiple of 64: lane
// (q16, g4) loads f = fb + 4 g4 .. fb + 4 g4 + 3 of its row, and k-step s of a 16-wide f block
// takes f = fb + 4 g4 + s (G is read in the same order, so the product is unchanged).  One
// wavefront per 64 rows x 64 columns starting at column 64 * blockIdx.y.  Two operand sets
// alternate (the next 16 columns are loaded while the current ones are multiplied); loads past
// d read column 0 with a zero weight, so they carry no branch.
__global__ __launch_bounds__(256) void k_dense_vec(int32_t n, int32_t d, int32_t B, const float* __restrict__ X,
                                                   const float* __restrict__ G, int32_t p0, int32_t bw, float alpha0,
                                                   float lambda, float* __restrict__ R0) {
    const int wave = (int)((blockIdx.x * 256u + threadIdx.x) >> 6);
    const int lane = threadIdx.x & 63, q16 = lane & 15, g4 = lane >> 4;
    const int qb = 64 * blockIdx.y;
    const int64_t r0 = (int64_t)wave * 64;
    if (r0 >= n) return;
    floatx4 acc[4][4];
#pragma unroll
    for (int rt = 0; rt < 4; ++rt)
#pragma unroll
        for (int t = 0; t < 4; ++t) acc[rt][t] = floatx4{0.f, 0.f, 0.f, 0.f};
    const float* xr[4];
#pragma unroll
    for (int rt = 0; rt < 4; ++rt) {
        const int64_t r = r0 + 16 * rt + q16;
        xr[rt] = X + (size_t)(r < n ? r : r0) * d + 4 * g4;  // rows past n: a valid row, never written
    }
    const float* gc = G + (size_t)(4 * g4) * B + qb + q16;
    floatx4 a0[4], a1[4];
    float b0[4][4], b1[4][4];
    float z0, z1;
    auto load = [&](int fb, floatx4* a, float (*b)[4], float& z) {
        const bool in = fb < d;
        const int f = in ? fb : 0;
#pragma unroll
        for (int rt = 0; rt < 4; ++rt) a[rt] = *reinterpret_cast<const floatx4*>(xr[rt] + f);
#pragma unroll
        for (int s = 0; s < 4; ++s)
#pragma unroll
            for (int t = 0; t < 4; ++t) b[s][t] = gc[(size_t)(f + s) * B + 16 * t];
        z = in ? 1.f : 0.f;
        __builtin_amdgcn_sched_barrier(0);  // keep the loads ahead of the next MFMA block
    };
    auto mma = [&](floatx4* a, float (*b)[4], float z) {
#pragma unroll
        for (int rt = 0; rt < 4; ++rt) a[rt] *= z;
#pragma unroll
        for (int s = 0; s < 4; ++s)
#pragma unroll
            for (int rt = 0; rt < 4; ++rt)
#pragma unroll
                for (int t = 0; t < 4; ++t) acc[rt][t] = mfma4(a[rt][s], b[s][t], acc[rt][t]);
    };
    load(0, a0, b0, z0);
    for (int fb = 0; fb < d; fb += 32) {
        load(fb + 16, a1, b1, z1);
        mma(a0, b0, z0);
        load(fb + 32, a0, b0, z0);
        mma(a1, b1, z1);
    }
#pragma unroll
    for (int rt = 0; rt < 4; ++rt)
#pragma unroll
        for (int t = 0; t < 4; ++t)
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int64_t r = r0 + 16 * rt + 4 * g4 + j;
                const int q = qb + 16 * t + q16;
                if (r < n)
                    R0[(size_t)r * B + q] =
                        (q < bw) ? fmaf(alpha0, acc[rt][t][j], lambda * X[(size_t)r * d + p0 + q]) : 0.f;
            }
}

// The same, with the G operand staged through LDS: the four wavefronts of a block take the
// same 64 columns of G (and 4 x 64 different rows of X), so each 16 x 64 slice of G is loaded
// once per block (one 16-byte load per thread) and read by every wavefront as 16-byte LDS reads
// (stored column-major at a pitch of 20 floats: lane (q16, g4) of tile t reads the four
// consecutive k-steps of column 16 t + q16; the k-step index of column c is XORed with
// 4 ((c / 16) mod 4), which spreads the 64 lanes of a staging store over all banks (without
// it they met 4-way conflicts) and keeps the tile reads spread: 27 M instead of 83 M conflict
// cycles per launch on the MSD-shaped W).  Two slices alternate: the next one is loaded
// while the current one is multiplied, one barrier per 16 columns of f.  Rows past n read row
// 0 and are never written.
// RT: row tiles of 16 per wavefront: 2 (32 rows, five wavefronts per SIMD; 64 rows at three
// per SIMD was 12 % slower for the d = 1024 user table and the same at d = 2048), or 1 for
// tables whose blocks of 256 rows would number fewer than two per CU, such as the item side
// at the MSD shape.
constexpr int kGsPitch = 20;
template <int RT>
__global__ __launch_bounds__(256) void k_dense_lds(int32_t n, int32_t d, int32_t B, const float* __restrict__ X,
                                                   const float* __restrict__ G, int32_t p0, int32_t bw, float alpha0,
                                                   float lambda, float* __restrict__ R0) {
    __shared__ __align__(16) float gs[2][64 * kGsPitch];
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63, q16 = lane & 15, g4 = lane >> 4;
    const int qb = 64 * blockIdx.y;
    const int64_t r0 = ((int64_t)blockIdx.x * 4 + wave) * (16 * RT);
    floatx4 acc[RT][4];
#pragma unroll
    for (int rt = 0; rt < RT; ++rt)
#pragma unroll
        for (int t = 0; t < 4; ++t) acc[rt][t] = floatx4{0.f, 0.f, 0.f, 0.f};
    const float* xr[RT];
#pragma unroll
    for (int rt = 0; rt < RT; ++rt) {
        const int64_t r = r0 + 16 * rt + q16;
        xr[rt] = X + (size_t)(r < n ? r : 0) * d + 4 * g4;
    }
    // staging: thread (row sr = tid / 16, quad sq = tid % 16) loads G[fb + sr][qb + 4 sq .. + 3]
    const int sr = tid >> 4, sq = tid & 15;
    const float* gsrc = G + (size_t)sr * B + qb + 4 * sq;
    auto gload = [&](int fb) {
        const int f = fb < d ? fb : 0;
        return *reinterpret_cast<const floatx4*>(gsrc + (size_t)f * B);
    };
    auto gstore = [&](int buf, floatx4 v) {
#pragma unroll
        for (int c = 0; c < 4; ++c) gs[buf][(4 * sq + c) * kGsPitch + (sr ^ (4 * (sq >> 2)))] = v[c];
    };
    auto xload = [&](int fb, floatx4* a) {
        const int f = fb < d ? fb : 0;
#pragma unroll
        for (int rt = 0; rt < RT; ++rt) a[rt] = *reinterpret_cast<const floatx4*>(xr[rt] + f);
    };
    auto mma = [&](int buf, const floatx4* a) {
        floatx4 b[4];
#pragma unroll
        for (int t = 0; t < 4; ++t)
            b[t] = *reinterpret_cast<const floatx4*>(&gs[buf][(16 * t + q16) * kGsPitch + 4 * (g4 ^ t)]);
#pragma unroll
        for (int s = 0; s < 4; ++s)
#pragma unroll
            for (int rt = 0; rt < RT; ++rt)
#pragma unroll
                for (int t = 0; t < 4; ++t) acc[rt][t] = mfma4(a[rt][s], b[t][s], acc[rt][t]);
    };
    floatx4 a0[RT], a1[RT];
    gstore(0, gload(0));
    xload(0, a0);
    __syncthreads();
    // d is a multiple of 32 here: two slices per iteration, no tail
    for (int fb = 0; fb < d; fb += 32) {
        const floatx4 g1 = gload(fb + 16);
        xload(fb + 16, a1);
        __builtin_amdgcn_sched_barrier(0);
        mma(0, a0);
        gstore(1, g1);
        __syncthreads();
        const floatx4 g0 = gload(fb + 32);
        xload(fb + 32, a0);
        __builtin_amdgcn_sched_barrier(0);
        mma(1, a1);
        gstore(0, g0);
        __syncthreads();
    }
    if (r0 >= n) return;
#pragma unroll
    for (int rt = 0; rt < RT; ++rt)
#pragma unroll
        for (int t = 0; t < 4; ++t)
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int64_t r = r0 + 16 * rt + 4 * g4 + j;
                const int q = qb + 16 * t + q16;
                if (r < n)
                    R0[(size_t)r * B + q] =
                        (q < bw) ? fmaf(alpha0, acc[rt][t][j], lambda * X[(size_t)r * d + p0 + q]) : 0.f;
            }
}

// ---- loss (eq. 2) in float64 ----

// Observed term sum_S alpha (<w_u,h_i> - y)^2 with the dot products in float64;
// one partial per wavefront (user).
__global__ __launch_bounds__(256) void k_loss_obs(int32_t U, int32_t d, const int64_t* __restrict__ ptr,
                                                  const int32_t* __restrict__ col, const float* __restrict__ y,
                                                  const float* __restrict__ a, const float* __restrict__ W,
                                                  const float* __restrict__ H, double* __restrict__ part) {
    const int u = (int)((blockIdx.x * 256u + threadIdx.x) >> 6);
    const int lane = threadIdx.x & 63, q16 = lane & 15, g4 = lane >> 4;
    if (u >= U) return;
    const float* w = W + (size_t)u * d;
    const int64_t lo = ptr[u], hi = ptr[u + 1];
    double acc = 0.0;
    for (int64_t k0 = lo; k0 < hi; k0 += 4) {
        const int64_t k = k0 + g4;
        const bool v = k < hi;
        const float* h = H + (size_t)(v ? col[k] : 0) * d;
        double s = 0.0;
        for (int f = q16; f < d; f += 16) s = fma((double)w[f], (double)h[f], s);
        s += __shfl_xor(s, 8);
        s += __shfl_xor(s, 4);
        s += __shfl_xor(s, 2);
        s += __shfl_xor(s, 1);
        if (v && q16 == 0) {
            const double e = s - (y ? (double)y[k] : 1.0);
            acc += (a ? (double)a[k] : 1.0) * e * e;
        }
    }
    acc += __shfl_xor(acc, 16);
    acc += __shfl_xor(acc, 32);
    if (lane == 0) part[u] = acc;
}

// Float64 Gramian partial: part[chunk][f][g] = sum_{r in chunk} X[r][f] X[r][g];
// 256 threads own a 64 x 64 output tile (4 x 4 per thread), X staged in LDS.
__global__ __launch_bounds__(256) void k_gram64_part(int32_t n, int32_t d, const float* __restrict__ X,
                                                     int32_t rows_per_chunk, double* __restrict__ part) {
    __shared__ double sf[32][64 + 1];
    __shared__ double sg[32][64 + 1];
    const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
    const int f0 = blockIdx.x * 64, g0 = blockIdx.y * 64, chunk = blockIdx.z;
    const int64_t r0 = (int64_t)chunk * rows_per_chunk;
    const int64_t r1 = std::min<int64_t>(n, r0 + rows_per_chunk);
    double acc[4][4] = {};
    for (int64_t rb = r0; rb < r1; rb += 32) {
        for (int e = threadIdx.x; e < 32 * 64; e += 256) {
            const int rr = e / 64, cc = e % 64;
            const int64_t r = rb + rr;
            sf[rr][cc] = (r < r1 && f0 + cc < d) ? (double)X[(size_t)r * d + f0 + cc] : 0.0;
            sg[rr][cc] = (r < r1 && g0 + cc < d) ? (double)X[(size_t)r * d + g0 + cc] : 0.0;
        }
        __syncthreads();
        for (int rr = 0; rr < 32; ++rr) {
            double xf[4], xg[4];
            for (int i = 0; i < 4; ++i) xf[i] = sf[rr][ty + 16 * i];
            for (int j = 0; j < 4; ++j) xg[j] = sg[rr][tx + 16 * j];
            for (int i = 0; i < 4; ++i)
                for (int j = 0; j < 4; ++j) acc[i][j] = fma(xf[i], xg[j], acc[i][j]);
        }
        __syncthreads();
    }
    double* out = part + (size_t)chunk * d * d;
    for (int i = 0; i < 4; ++i)
        for (int j = 0; j < 4; ++j) {
            const int f = f0 + ty + 16 * i, g = g0 + tx + 16 * j;
            if (f < d && g < d) out[(size_t)f * d + g] = acc[i][j];
        }
}

__global__ void k_gram64_reduce(const double* __restrict__ part, int32_t nchunks, int64_t count,
                                double* __restrict__ out) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= count) return;
    double s = 0.0;
    for (int c = 0; c < nchunks; ++c) s += part[(size_t)c * count + e];
    out[e] = s;
}

// out[0] = observed term, out[1] = <GW, GH>_F, out[2] = tr GW + tr GH (one block, fixed order).
__global__ __launch_bounds__(256) void k_loss_combine(const double* __restrict__ obs_part, int64_t nobs,
                                                      const double* __restrict__ GW, const double* __restrict__ GH,
                                                      int32_t d, double* __restrict__ out) {
    __shared__ double red[3][256];
    double s0 = 0.0, s1 = 0.0, s2 = 0.0;
    for (int64_t e = threadIdx.x; e < nobs; e += 256) s0 += obs_part[e];
    const int64_t dd = (int64_t)d * d;
    for (int64_t e = threadIdx.x; e < dd; e += 256) s1 += GW[e] * GH[e];
    for (int64_t f = threadIdx.x; f < d; f += 256) s2 += GW[f * d + f] + GH[f * d + f];
    red[0][threadIdx.x] = s0;
    red[1][threadIdx.x] = s1;
    red[2][threadIdx.x] = s2;
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off)
            for (int k = 0; k < 3; ++k) red[k][threadIdx.x] += red[k][threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x < 3) out[threadIdx.x] = red[threadIdx.x][0];
}

int chunk_rows_for(int64_t n, int64_t tiles, int64_t target_blocks, int64_t min_rows) {
    int64_t chunks = std::max<int64_t>(1, target_blocks / std::max<int64_t>(tiles, 1));
    int64_t rows = (n + chunks - 1) / chunks;
    rows = std::max<int64_t>(rows, min_rows);
    rows = (rows + 3) / 4 * 4;
    return (int)std::max<int64_t>(rows, 4);
}

}  // namespace

namespace {
// p[e] = v for e < n (a kernel rather than a memset node, so that it can be captured in graphs)
__global__ __launch_bounds__(256) void k_fill_f32(float* __restrict__ p, int64_t n, float v) {
    const int64_t e0 = ((int64_t)blockIdx.x * 256 + threadIdx.x) * 4;
    const int64_t stride = (int64_t)gridDim.x * 256 * 4;
    for (int64_t e = e0; e < n; e += stride) {
        if (e + 4 <= n && (reinterpret_cast<uintptr_t>(p + e) & 15u) == 0)
            *reinterpret_cast<float4*>(p + e) = make_float4(v, v, v, v);
        else
            for (int64_t j = e; j < std::min<int64_t>(n, e + 4); ++j) p[j] = v;
    }
}
}  // namespace

void launch_fill(hipStream_t st, float* p, int64_t n, float v) {
    if (n <= 0) return;
    const int64_t blocks = std::min<int64_t>(8192, (n + 1023) / 1024);
    hipLaunchKernelGGL(k_fill_f32, dim3((unsigned)blocks), dim3(256), 0, st, p, n, v);
}

void launch_gram_reduce(hipStream_t st, const float* part, int32_t nchunks, int64_t count, float* out) {
    hipLaunchKernelGGL(k_gram_reduce, dim3(nblk(count, 16)), dim3(256), 0, st, part, nchunks, count, out);
}

size_t gram_part_floats_needed(int32_t n, int32_t d, int32_t ncols, bool bf16) {
    const int64_t tiles = (int64_t)((d + 63) / 64) * ((ncols + 63) / 64);
    const int rows = chunk_rows_for(n, tiles, 2048, 64);
    const int64_t chunks = (n + rows - 1) / rows;
    size_t need = (size_t)std::max<int64_t>(chunks, 1) * d * ncols;
    if (bf16 && ncols == d && d % kGLT == 0)
        need = std::max(need, (size_t)gram_lds_chunks(n, d) * gram_lds_tiles(d) * kGLTileFloats);
    return need;
}

// inside == false: c->yhat becomes the cache relative to block blk; inside == true:
// out = c->yhat + the block's part (the predictions themselves).
void launch_predict(ials_ctx* c, int32_t blk, bool inside, float* out) {
    const SideIndex& us = c->side[IALS_SIDE_USER];
    if (c->U == 0 || c->nnz == 0) return;
    const int32_t p0 = blk * c->b, bw = std::min(c->b, c->d - p0);
    const unsigned g = nblk(c->U, 4);
    // the specialised kernels read rows with 16-byte loads
    const bool aligned = reinterpret_cast<uintptr_t>(c->W) % 16 == 0 && reinterpret_cast<uintptr_t>(c->H) % 16 == 0;
    if (!aligned) {
        hipLaunchKernelGGL(k_predict, dim3(g), dim3(256), 0, c->stream, c->U, c->d, us.ptr, us.col, c->W, c->H, p0, bw,
                           inside, c->yhat, out);
    } else if (c->d == 64 || c->d == 128 || c->d == 256) {
        // the 64-column chunks that hold at least one summed column
        int chs[4] = {0, 0, 0, 0}, nc = 0;
        for (int j = 0; j < c->d / 64; ++j) {
            bool any = false;
            for (int f = 64 * j; f < 64 * j + 64; ++f) any = any || ((f >= p0 && f < p0 + bw) == inside);
            if (any) chs[nc++] = j;
        }
        if (nc == 0) chs[nc++] = 0;  // nothing summed: one masked chunk keeps the output defined
        const int4 ch = make_int4(chs[0], chs[1], chs[2], chs[3]);
#define IALS_PRED(JV, JLV)                                                                                     \
    hipLaunchKernelGGL((k_predict_rows<JV, JLV>), dim3(g), dim3(256), 0, c->stream, c->U, us.ptr, us.col, c->W, \
                       c->H, p0, bw, inside, ch, c->yhat, out)
        if (c->d == 64) IALS_PRED(1, 1);
        else if (c->d == 128) {
            if (nc == 1) IALS_PRED(2, 1);
            else IALS_PRED(2, 2);
        } else {
            if (nc == 1) IALS_PRED(4, 1);
            else if (nc == 2) IALS_PRED(4, 2);
            else if (nc == 3) IALS_PRED(4, 3);
            else IALS_PRED(4, 4);
        }
#undef IALS_PRED
    } else if (c->d == 512)
        hipLaunchKernelGGL((k_predict_wide<2, 4>), dim3(g), dim3(256), 0, c->stream, c->U, us.ptr, us.col, c->W, c->H,
                           p0, bw, inside, c->yhat, out);
    else if (c->d == 1024)
        hipLaunchKernelGGL((k_predict_wide<4, 4>), dim3(g), dim3(256), 0, c->stream, c->U, us.ptr, us.col, c->W, c->H,
                           p0, bw, inside, c->yhat, out);
    else if (c->d == 2048) {
        // two slices of 1,024 columns: 168 MB of H per slice at the MSD shape; eight
        // observations' rows in flight per wavefront
        for (int f0 = 0; f0 < 2048; f0 += 1024)
            hipLaunchKernelGGL((k_predict_slice<4, 8>), dim3(g), dim3(256), 0, c->stream, c->U, c->d, f0, f0 == 0,
                               us.ptr, us.col, c->W, c->H, p0, bw, inside, c->yhat, out);
    }
    else
        hipLaunchKernelGGL(k_predict, dim3(g), dim3(256), 0, c->stream, c->U, c->d, us.ptr, us.col, c->W, c->H, p0, bw,
                           inside, c->yhat, out);
}

// out (d x ncols) = X^T X[:, p0:p0+bw] (zero columns for q >= bw).
void launch_gramian_raw(hipStream_t st, const float* X, int32_t n, int32_t d, int32_t p0, int32_t bw, int32_t ncols,
                        float* part, float* out, bool bf16, int32_t split) {
    const int64_t ft = (d + 63) / 64;
    const int qt16 = (ncols + 15) / 16;
    const int QT = qt16 >= 4 ? 4 : (qt16 >= 2 ? 2 : 1);
    const int64_t qg = (ncols + 16 * QT - 1) / (16 * QT);
    const int rows = chunk_rows_for(n, ft * qg, 2048, 64);
    const int64_t chunks = std::max<int64_t>(1, (n + rows - 1) / rows);
    dim3 grid((unsigned)ft, (unsigned)qg, (unsigned)chunks);
    if (bf16 && p0 == 0 && bw == d && ncols == d && d % kGLT == 0 && reinterpret_cast<uintptr_t>(X) % 16 == 0 &&
        ((int64_t)n + 2 * kGLK) * d * 4 < ((int64_t)1 << 31)) {
        // the full Gramian: LDS-staged 256 x 256 lower tiles, partials summed in float64
        const int tiles = gram_lds_tiles(d), nch = gram_lds_chunks(n, d);
        int64_t rows = (n + nch - 1) / nch;
        rows = std::max<int64_t>(kGLK, (rows + kGLK - 1) / kGLK * kGLK);
        const int per_xcd = (tiles * nch + 7) / 8;
        static OccCache occ;
        (void)resident_per_cu(occ, reinterpret_cast<const void*>(&k_gram_bf16_lds), 512, kGLLds, true, 1);
        hipLaunchKernelGGL(k_gram_bf16_lds, dim3((unsigned)(8 * per_xcd)), dim3(512), kGLLds, st, n, d, X, tiles, nch,
                           per_xcd, (int32_t)rows, part);
        hipLaunchKernelGGL(k_gram_lds_reduce, dim3(nblk((int64_t)tiles * kGLTileFloats, 256)), dim3(256), 0, st, part,
                           tiles, nch, d, out);
        return;
    }
    if (d % 64 == 0 && ncols % 64 == 0 && bw == ncols && p0 % 4 == 0 && reinterpret_cast<uintptr_t>(X) % 16 == 0) {
        // full 64 x 64 tiles with 16-byte loads; four wavefronts per block, so a quarter of the
        // blocks (and of the partials the reduction reads) for the same number of wavefronts
        const int rv = chunk_rows_for(n, ft * qg, split, 256);
        const int64_t cv = std::max<int64_t>(1, (n + rv - 1) / rv);
        if (bf16)
            hipLaunchKernelGGL(k_gram_vec_bf16, dim3((unsigned)ft, (unsigned)qg, (unsigned)cv), dim3(256), 0, st, n, d,
                               X, p0, ncols, rv, part);
        else if (((int64_t)rv + 160) * d * 4 < ((int64_t)1 << 31))
            hipLaunchKernelGGL(k_gram_buf, dim3((unsigned)ft, (unsigned)qg, (unsigned)cv), dim3(256), 0, st, n, d, X,
                               p0, ncols, rv, part);
        else
            hipLaunchKernelGGL(k_gram_vec, dim3((unsigned)ft, (unsigned)qg, (unsigned)cv), dim3(256), 0, st, n, d, X,
                               p0, ncols, rv, part);
        const int64_t count = (int64_t)d * ncols;
        hipLaunchKernelGGL(k_gram_reduce, dim3(nblk(count, 16)), dim3(256), 0, st, part, (int32_t)cv, count, out);
        return;
    }
#define IALS_GRAM(Q, BFV) hipLaunchKernelGGL((k_gram_part<Q, BFV>), grid, dim3(64), 0, st, n, d, X, p0, bw, ncols, rows, part)
    if (bf16) {
        if (QT == 4) IALS_GRAM(4, true);
        else if (QT == 2) IALS_GRAM(2, true);
        else IALS_GRAM(1, true);
    } else {
        if (QT == 4) IALS_GRAM(4, false);
        else if (QT == 2) IALS_GRAM(2, false);
        else IALS_GRAM(1, false);
    }
#undef IALS_GRAM
    const int64_t count = (int64_t)d * ncols;
    hipLaunchKernelGGL(k_gram_reduce, dim3(nblk(count, 16)), dim3(256), 0, st, part, (int32_t)chunks, count, out);
}

// The same on the context's stream and scratch; with make_dmat also forms Dmat for
// the pass and resets the sweep cursors.
void launch_gramian_slab(ials_ctx* c, const float* X, int32_t n, int32_t p0, int32_t bw, int32_t ncols, float* out,
                         bool make_dmat) {
    launch_gramian_raw(c->stream, X, n, c->d, p0, bw, ncols, c->gram_part, out, c->precision == IALS_PREC_BF16,
                       c->gram_split);
    if (make_dmat)
        hipLaunchKernelGGL(k_make_dmat, dim3(nblk(std::max(c->B * c->B, (int)CUR_NUM), 256)), dim3(256), 0, c->stream,
                           out, c->B, p0, bw, c->alpha0, c->lambda, c->Dmat, c->cursors);
}

void launch_dense(ials_ctx* c, const float* X, int32_t n, int32_t p0, int32_t bw) {
    if (n == 0) return;
    const unsigned grid = nblk(n, 256);  // blocks of 4 waves x 64 rows
    const int B = c->B;
    if (B % 64 == 0 && c->d % 32 == 0 && reinterpret_cast<uintptr_t>(X) % 16 == 0 &&
        reinterpret_cast<uintptr_t>(c->G) % 16 == 0) {
        if ((int64_t)grid * (B / 64) >= 2 * (int64_t)c->num_cu)
            hipLaunchKernelGGL((k_dense_lds<2>), dim3(nblk(n, 128), (unsigned)(B / 64)), dim3(256), 0, c->stream, n,
                               c->d, B, X, c->G, p0, bw, c->alpha0, c->lambda, c->R0);
        else
            hipLaunchKernelGGL((k_dense_lds<1>), dim3(nblk(n, 64), (unsigned)(B / 64)), dim3(256), 0, c->stream, n, c->d,
                               B, X, c->G, p0, bw, c->alpha0, c->lambda, c->R0);
        return;
    }
    if (B % 64 == 0 && c->d % 16 == 0 && reinterpret_cast<uintptr_t>(X) % 16 == 0) {
        hipLaunchKernelGGL(k_dense_vec, dim3(grid, (unsigned)(B / 64)), dim3(256), 0, c->stream, n, c->d, B, X, c->G, p0,
                           bw, c->alpha0, c->lambda, c->R0);
        return;
    }
#define IALS_DENSE(NTV, GY)                                                                                      \
    hipLaunchKernelGGL(k_dense<NTV>, dim3(grid, GY), dim3(256), 0, c->stream, n, c->d, B, X, c->G, p0, bw,       \
                       c->alpha0, c->lambda, c->R0)
    switch (B) {
        case 16: IALS_DENSE(1, 1); break;
        case 32: IALS_DENSE(2, 1); break;
        case 48: IALS_DENSE(3, 1); break;
        default: IALS_DENSE(4, (unsigned)(B / 64)); break;
    }
#undef IALS_DENSE
}

ials_status launch_loss(ials_ctx* c) {
    hipStream_t st = c->stream;
    const int32_t d = c->d;
    const SideIndex& us = c->side[IALS_SIDE_USER];
    if (c->U > 0)
        hipLaunchKernelGGL(k_loss_obs, dim3(nblk(c->U, 4)), dim3(256), 0, st, c->U, d, us.ptr, us.col, us.y, us.a, c->W,
                           c->H, c->loss_part);
    // float64 Gramians; partials reuse the loss scratch after the observed partials
    double* part = c->loss_part + std::max<int64_t>(c->U, 1);
    const size_t part_cap = c->loss_part_len - (size_t)std::max<int64_t>(c->U, 1);
    const int64_t tiles = (int64_t)((d + 63) / 64) * ((d + 63) / 64);
    for (int m = 0; m < 2; ++m) {
        const float* X = m == 0 ? c->W : c->H;
        const int64_t n = m == 0 ? c->U : c->I;
        const int64_t max_chunks = std::max<int64_t>(1, (int64_t)(part_cap / ((size_t)d * d)));
        int64_t chunks = std::min<int64_t>(max_chunks, std::max<int64_t>(1, 2048 / tiles));
        int64_t rows = (n + chunks - 1) / chunks;
        rows = std::max<int64_t>(rows, 32);
        chunks = std::max<int64_t>(1, (n + rows - 1) / rows);
        dim3 grid((unsigned)((d + 63) / 64), (unsigned)((d + 63) / 64), (unsigned)chunks);
        hipLaunchKernelGGL(k_gram64_part, grid, dim3(256), 0, st, (int32_t)n, d, X, (int32_t)rows, part);
        const int64_t count = (int64_t)d * d;
        hipLaunchKernelGGL(k_gram64_reduce, dim3(nblk(count, 256)), dim3(256), 0, st, part, (int32_t)chunks, count,
                           c->gram64 + (size_t)m * count);
    }
    hipLaunchKernelGGL(k_loss_combine, dim3(1), dim3(256), 0, st, c->loss_part, (int64_t)c->U, c->gram64,
                       c->gram64 + (size_t)d * d, d, c->loss_out);
    IALS_HIP_TRY(c, hipGetLastError());
    return IALS_OK;
}

}  // namespace ials
