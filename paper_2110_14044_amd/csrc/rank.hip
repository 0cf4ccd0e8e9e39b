// Top-k recommendation and its ranking metrics (gfx950, wave64).
//
// Items are ranked for a user by the score of matrix factorisation, yhat(u, i) = <w_u, h_i>
// (sec. 2, eq. 1); the evaluation of sec. 5.1 ranks all items not given for a user and
// measures Recall@k and NDCG@k against the held-out ones.
//
//   k_score       S = W H^T for a batch of users, MFMA f32 16x16x4: a wavefront forms a 64 items x
//                 64 users tile from 16-byte loads along f (the reduction index taken in the same
//                 permuted order in both operands), items as the A operand so that each lane ends
//                 with four consecutive items of one user and stores them as one 16-byte store
//   k_mask_excl   S[u][i] = -inf for the items excluded for u (its fold-in / training items)
//   k_select      one wavefront per user: a histogram of an eighth of the row (every eighth run of
//                 64 float4s) places a threshold that about 2k items should clear, and one pass
//                 collects those into LDS; when fewer than k or more than the buffer clear it, an
//                 MSB-first radix select on the order-preserving integer key of the scores (digits
//                 of 11, 11 and 10 bits, histograms in LDS) runs until the items at or above the
//                 current bucket fit the LDS candidate buffer, and one more pass collects them.
//                 A bitonic sort in LDS orders the candidates by (score desc, id asc); exact ties
//                 beyond the buffer are taken in ascending id order
//   k_rank_metrics / k_metric_sums
//                 Recall@k and NDCG@k per user in float64 (held-out lists searched by bisection),
//                 then their sums over users in a fixed order
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <mutex>
#include <string>

#include "ials.h"

// Score buffer of ials_rank_topk_noalloc: a fixed array in device memory, one copy per GPU
// the library runs on, held until the process ends.  Host code never passes its name to a
// kernel (on the host it is only a stand-in for the symbol): it takes the device address
// from hipGetSymbolAddress once per device and passes that.
constexpr size_t kRankScratchBytes = size_t(64) << 20;
static __device__ __align__(256) float scratch[kRankScratchBytes / sizeof(float)];

namespace {

typedef float floatx4_r __attribute__((ext_vector_type(4)));

thread_local std::string g_rank_error;

ials_status rank_fail(ials_status s, const std::string& msg) {
    g_rank_error = msg;
    return s;
}

__device__ inline floatx4_r mfma16x4(float a, float b, floatx4_r c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

__device__ inline void lds_sync_wave() {
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
    __builtin_amdgcn_wave_barrier();
}

// order-preserving map of a float to an unsigned key (larger float, larger key); -0 and +0
// share the key of +0, as they compare equal
__device__ inline uint32_t fkey(float f) {
    const uint32_t b = f == 0.f ? 0u : __float_as_uint(f);
    return (b & 0x80000000u) ? ~b : (b | 0x80000000u);
}
__device__ inline float fval(uint32_t k) {
    return __uint_as_float((k & 0x80000000u) ? (k & 0x7fffffffu) : ~k);
}

// ---------------------------------------------------------------------------------------------
// S[u - u0][i] = <w_u, h_i> for u in [u0, u0 + nu), i in [0, I4) (-inf for i >= I), row pitch I4.
// Workgroup: 4 wavefronts in 2 x 2, 128 items x 128 users; wavefront: 4 x 4 tiles of 16 x 16.
// The grid is one-dimensional: 8 ipx n_ut workgroups for n_ut user tiles and ipx = ceil(n_it / 8).
// Per 16 columns of f, lane (q = l % 16, g = l / 16) loads f in [f0 + 4g, f0 + 4g + 4) of 4 item
// rows and 4 user rows and feeds component s to the MFMA k slot g of step s, in both operands.
__global__ __launch_bounds__(256) void k_score(const float* __restrict__ W, const float* __restrict__ H, int32_t d,
                                               int64_t u0, int32_t nu, int32_t I, int32_t I4,
                                               float* __restrict__ S) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, q = lane & 15, g = lane >> 4;
    // Workgroups are dealt to the 8 XCDs round-robin (workgroup w runs on XCD w % 8); XCD x takes
    // the item tiles [x ipx, (x + 1) ipx) for every user tile, so that its L2 holds 1/8 of H.
    const int n_it = (I4 + 127) / 128, ipx = (n_it + 7) / 8;
    const int w = blockIdx.x, xcd = w & 7, l = w >> 3;
    const int it = xcd * ipx + l % ipx, ut = l / ipx;
    if (it >= n_it || ut * 128 >= nu) return;  // padding workgroups of the last XCDs' ranges
    const int i_base = it * 128 + (wave & 1) * 64;
    const int u_base = ut * 128 + (wave >> 1) * 64;
    const float* hr[4];
    const float* wr[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        const int i = std::min(i_base + 16 * t + q, I - 1);
        const int u = std::min(u_base + 16 * t + q, nu - 1);
        hr[t] = H + (size_t)i * d;
        wr[t] = W + (size_t)(u0 + u) * d;
    }
    floatx4_r acc[4][4];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) acc[a][b] = floatx4_r{0.f, 0.f, 0.f, 0.f};
    // Two sets of operands alternate: the next 16 columns are loaded while the current 16 are
    // multiplied.  The loads have no branches (columns past d read column 0, and their item
    // operand is zeroed where it is used), and the sets are never copied, so that waiting for
    // the current operands does not also wait for the ones in flight.
    floatx4_r a0[4], b0[4], a1[4], b1[4];
    float z0, z1;
    auto load = [&](int f0, floatx4_r* av, floatx4_r* bv, float& z) {
        const int f = f0 + 4 * g;
        const bool in = f < d;  // d is a multiple of 4
        const int fc = in ? f : 0;
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            av[t] = *reinterpret_cast<const floatx4_r*>(hr[t] + fc);
            bv[t] = *reinterpret_cast<const floatx4_r*>(wr[t] + fc);
        }
        z = in ? 1.f : 0.f;
        __builtin_amdgcn_sched_barrier(0);  // keep the loads ahead of the next MFMA block
    };
    auto mma = [&](floatx4_r* av, const floatx4_r* bv, float z) {
#pragma unroll
        for (int t = 0; t < 4; ++t) av[t] *= z;
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
            for (int b = 0; b < 4; ++b) {
                acc[a][b] = mfma16x4(av[a][0], bv[b][0], acc[a][b]);
                acc[a][b] = mfma16x4(av[a][1], bv[b][1], acc[a][b]);
                acc[a][b] = mfma16x4(av[a][2], bv[b][2], acc[a][b]);
                acc[a][b] = mfma16x4(av[a][3], bv[b][3], acc[a][b]);
            }
    };
    load(0, a0, b0, z0);
    for (int f0 = 0; f0 < d; f0 += 32) {
        load(f0 + 16, a1, b1, z1);
        mma(a0, b0, z0);
        load(f0 + 32, a0, b0, z0);
        mma(a1, b1, z1);
    }
    // accumulator layout: lane l, register j = (item row 4 g + j, user column q) of the tile
#pragma unroll
    for (int b = 0; b < 4; ++b) {
        const int u = u_base + 16 * b + q;
        if (u >= nu) continue;
        float* srow = S + (size_t)u * I4;
#pragma unroll
        for (int a = 0; a < 4; ++a) {
            const int i = i_base + 16 * a + 4 * g;
            if (i >= I4) continue;
            floatx4_r v;
#pragma unroll
            for (int j = 0; j < 4; ++j) v[j] = (i + j < I) ? acc[a][b][j] : -INFINITY;
            *reinterpret_cast<floatx4_r*>(srow + i) = v;
        }
    }
}

// S[u - u0][i] = -inf for every excluded item i of user u (ids outside [0, I) are ignored).
// One wavefront per user.
__global__ __launch_bounds__(256) void k_mask_excl(const int64_t* __restrict__ ptr, const int32_t* __restrict__ idx,
                                                   int64_t u0, int32_t nu, int32_t I, int32_t I4, float* __restrict__ S) {
    const int u = (int)((blockIdx.x * 256u + threadIdx.x) >> 6), lane = threadIdx.x & 63;
    if (u >= nu) return;
    const int64_t lo = ptr[u0 + u], hi = ptr[u0 + u + 1];
    float* srow = S + (size_t)u * I4;
    for (int64_t e = lo + lane; e < hi; e += 64) {
        const int i = idx[e];
        if (i >= 0 && i < I) srow[i] = -INFINITY;
    }
}

constexpr int kSelCap = 1024;  // LDS candidates per wavefront
constexpr int kSelBins = 2048;
constexpr int kMaxK = 512;

// The histogram is needed only before the candidates are collected, so the two share storage.
struct SelLds {
    union {
        uint32_t bins[kSelBins];
        struct {
            uint32_t key[kSelCap];
            int32_t id[kSelCap];
        } c;
    };
    uint32_t lane_sum[64];
};
static_assert(sizeof(SelLds) * 4 <= 40 * 1024, "four wavefronts' selection state fits 40 KB of LDS");

// Exclusive count of set bits of m below this lane.
__device__ inline int lanes_below(uint64_t m) {
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0));
}

// Scores of items 4 (t0 + 64 r + lane) + j (r, j < 4) of a row: four 16-byte loads in flight per
// lane (-inf past the row); e[4 r + j].
__device__ inline void load_row16(const float* srow, int n4, int t0, int lane, float (&e)[16]) {
    floatx4_r v[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int t = t0 + 64 * r + lane;
        v[r] = t < n4 ? __builtin_nontemporal_load(reinterpret_cast<const floatx4_r*>(srow) + t)
                      : floatx4_r{-INFINITY, -INFINITY, -INFINITY, -INFINITY};
    }
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int j = 0; j < 4; ++j) e[4 * r + j] = v[r][j];
}

// Radix select of the k largest of a row, then their collection: see the file comment.  The
// candidates land in L.c (at most kSelCap); returns their number.
__device__ int radix_collect(SelLds& L, const float* srow, int n4, int I4, int k, int lane) {
    uint32_t prefix = 0, pmask = 0;  // fixed high bits of the key and their mask
    int need = k;                    // items still to select inside the current bucket
    int chosen = 0;                  // items already known to be in the top k (above the bucket)
    uint32_t lower = 0;              // collect every eligible item with key >= lower
    bool take_all = false, ties = false;
    for (int level = 0; level < 3; ++level) {
        const int shift = level == 0 ? 21 : (level == 1 ? 10 : 0);
        const int nbits = level == 2 ? 10 : 11;
        const uint32_t dmask = (1u << nbits) - 1u;
        const int nb = 1 << nbits;
        for (int b = lane; b < nb; b += 64) L.bins[b] = 0;
        lds_sync_wave();
        for (int t0 = 0; t0 < n4; t0 += 256) {
            float e[16];
            load_row16(srow, n4, t0, lane, e);
#pragma unroll
            for (int c = 0; c < 16; ++c) {
                const uint32_t key = fkey(e[c]);
                if (e[c] > -INFINITY && (key & pmask) == prefix) atomicAdd(&L.bins[(key >> shift) & dmask], 1u);
            }
        }
        lds_sync_wave();
        // per-lane sums of its bins, then the bin holding the need-th largest
        const int per = nb / 64;
        uint32_t s = 0;
        for (int b = 0; b < per; ++b) s += L.bins[lane * per + b];
        L.lane_sum[lane] = s;
        lds_sync_wave();
        uint32_t above_lane = 0, total = 0;
        for (int l = 0; l < 64; ++l) {
            const uint32_t x = L.lane_sum[l];
            total += x;
            if (l > lane) above_lane += x;
        }
        if ((int)total < need) {  // fewer eligible items than k (only possible at the first level)
            take_all = true;
            break;
        }
        int T = -1;
        uint32_t aboveT = 0, cntT = 0;
        if ((int)above_lane < need && (int)(above_lane + s) >= need) {
            uint32_t acc = above_lane;
            for (int b = per - 1; b >= 0; --b) {
                const uint32_t c = L.bins[lane * per + b];
                if ((int)(acc + c) >= need) {
                    T = lane * per + b;
                    aboveT = acc;
                    cntT = c;
                    break;
                }
                acc += c;
            }
        }
        const uint64_t found = __ballot(T >= 0);
        const int src = __builtin_ctzll(found);
        T = __shfl(T, src);
        aboveT = __shfl(aboveT, src);
        cntT = __shfl(cntT, src);
        lds_sync_wave();
        const uint32_t bucket = prefix | ((uint32_t)T << shift);
        if (chosen + (int)aboveT + (int)cntT <= kSelCap) {
            lower = bucket;
            break;
        }
        chosen += (int)aboveT;
        need -= (int)aboveT;
        prefix = bucket;
        pmask |= dmask << shift;
        if (level == 2) ties = true;  // the whole key is fixed: cntT > kSelCap - chosen equal keys
    }

    // collect
    int count = 0;
    if (!ties) {
        for (int t0 = 0; t0 < n4; t0 += 256) {
            float e[16];
            load_row16(srow, n4, t0, lane, e);
#pragma unroll
            for (int c = 0; c < 16; ++c) {
                const uint32_t key = fkey(e[c]);
                const bool take = e[c] > -INFINITY && (take_all || key >= lower);
                const uint64_t m = __ballot(take);
                const int pos = count + lanes_below(m);
                if (take && pos < kSelCap) {  // always true: the bucket was chosen to fit
                    L.c.key[pos] = key;
                    L.c.id[pos] = 4 * (t0 + 64 * (c >> 2) + lane) + (c & 3);
                }
                count = std::min(kSelCap, count + (int)__popcll(m));
            }
        }
    } else {
        // keys above the tie key (fewer than k), then equal keys in ascending id order up to k
        const uint32_t tk = prefix;
        for (int t0 = 0; t0 < n4; t0 += 256) {
            float e[16];
            load_row16(srow, n4, t0, lane, e);
#pragma unroll
            for (int c = 0; c < 16; ++c) {
                const uint32_t key = fkey(e[c]);
                const bool take = e[c] > -INFINITY && key > tk;
                const uint64_t m = __ballot(take);
                const int pos = count + lanes_below(m);
                if (take && pos < k) {  // always true: fewer than k keys lie above the tie key
                    L.c.key[pos] = key;
                    L.c.id[pos] = 4 * (t0 + 64 * (c >> 2) + lane) + (c & 3);
                }
                count = std::min(k, count + (int)__popcll(m));
            }
        }
        for (int i0 = 0; i0 < I4 && count < k; i0 += 64) {
            const int i = i0 + lane;
            const float e = i < I4 ? srow[i] : -INFINITY;
            const bool tie = e > -INFINITY && fkey(e) == tk;
            const uint64_t m = __ballot(tie);
            const int pos = count + lanes_below(m);
            if (tie && pos < k) {
                L.c.key[pos] = tk;
                L.c.id[pos] = i;
            }
            count = std::min(k, count + (int)__popcll(m));
        }
    }
    return count;
}

// Sampled threshold: the histogram of every eighth run of 64 float4s of the row places a key
// that about 2k items should clear (at most 3/4 of the candidate buffer); one pass collects
// every eligible item at or above it.  Returns the number collected when it is at least k and
// fits the buffer (then the collected items hold the top k), else -1.
__device__ int sampled_collect(SelLds& L, const float* srow, int n4, int k, int lane) {
    if (n4 == 0) return -1;
    for (int b = lane; b < kSelBins; b += 64) L.bins[b] = 0;
    lds_sync_wave();
    for (int t0 = 0; t0 < n4; t0 += 512) {
        const int t = t0 + lane;
        const floatx4_r v = t < n4 ? __builtin_nontemporal_load(reinterpret_cast<const floatx4_r*>(srow) + t)
                                   : floatx4_r{-INFINITY, -INFINITY, -INFINITY, -INFINITY};
#pragma unroll
        for (int j = 0; j < 4; ++j)
            if (v[j] > -INFINITY) atomicAdd(&L.bins[fkey(v[j]) >> 21], 1u);
    }
    lds_sync_wave();
    constexpr int per = kSelBins / 64;
    uint32_t s = 0;
    for (int b = 0; b < per; ++b) s += L.bins[lane * per + b];
    L.lane_sum[lane] = s;
    lds_sync_wave();
    uint32_t above_lane = 0, total = 0;
    for (int l = 0; l < 64; ++l) {
        const uint32_t x = L.lane_sum[l];
        total += x;
        if (l > lane) above_lane += x;
    }
    // sample items above the threshold: the target count scaled by the sampled fraction
    const int64_t target = std::min(2 * k, 3 * kSelCap / 4);
    const int m = (int)std::max<int64_t>(1, (target * (int64_t)total + 4ll * n4 - 1) / (4ll * n4));
    int T = 0;
    if ((int)total >= m) {
        int t_l = -1;
        if ((int)above_lane < m && (int)(above_lane + s) >= m) {
            uint32_t acc = above_lane;
            for (int b = per - 1; b >= 0; --b) {
                acc += L.bins[lane * per + b];
                if ((int)acc >= m) {
                    t_l = lane * per + b;
                    break;
                }
            }
        }
        const uint64_t found = __ballot(t_l >= 0);
        T = __shfl(t_l, __builtin_ctzll(found));
    }
    lds_sync_wave();  // the bins are read before the candidates overwrite them
    const uint32_t lower = (uint32_t)T << 21;
    int count = 0;
    for (int t0 = 0; t0 < n4; t0 += 256) {
        float e[16];
        load_row16(srow, n4, t0, lane, e);
#pragma unroll
        for (int c = 0; c < 16; ++c) {
            const uint32_t key = fkey(e[c]);
            const bool take = e[c] > -INFINITY && key >= lower;
            const uint64_t mk = __ballot(take);
            const int pos = count + lanes_below(mk);
            if (take && pos < kSelCap) {
                L.c.key[pos] = key;
                L.c.id[pos] = 4 * (t0 + 64 * (c >> 2) + lane) + (c & 3);
            }
            count += (int)__popcll(mk);
        }
    }
    lds_sync_wave();
    return (count >= k && count <= kSelCap) ? count : -1;
}

// One wavefront per user of the batch; see the file comment.
__global__ __launch_bounds__(256) void k_select(const float* __restrict__ S, int32_t nu, int32_t I4, int32_t k,
                                                int64_t u0, int32_t* __restrict__ out_ids, float* __restrict__ out_sc) {
    __shared__ SelLds lds_all[4];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int u = blockIdx.x * 4 + wave;
    if (u >= nu) return;  // wave-uniform; no workgroup barriers below
    SelLds& L = lds_all[wave];
    const float* srow = S + (size_t)u * I4;
    const int n4 = I4 / 4;

    int count = sampled_collect(L, srow, n4, k, lane);
    if (count < 0) count = radix_collect(L, srow, n4, I4, k, lane);
    lds_sync_wave();

    // bitonic sort of the candidates: descending key, ascending id; padding (key 0) sorts last
    int n2 = 1;
    while (n2 < count) n2 <<= 1;
    for (int p = count + lane; p < n2; p += 64) {
        L.c.key[p] = 0;
        L.c.id[p] = 0x7fffffff;
    }
    lds_sync_wave();
    for (int size = 2; size <= n2; size <<= 1) {
        for (int stride = size >> 1; stride > 0; stride >>= 1) {
            for (int p = lane; p < n2 / 2; p += 64) {
                const int i = 2 * stride * (p / stride) + (p % stride);
                const int j = i + stride;
                const uint32_t ki = L.c.key[i], kj = L.c.key[j];
                const int32_t ii = L.c.id[i], ij = L.c.id[j];
                // does j come before i in the final (descending) order?
                const bool j_first = kj > ki || (kj == ki && ij < ii);
                const bool desc = (i & size) == 0;
                if (desc ? j_first : !j_first) {
                    L.c.key[i] = kj;
                    L.c.key[j] = ki;
                    L.c.id[i] = ij;
                    L.c.id[j] = ii;
                }
            }
            lds_sync_wave();
        }
    }
    int32_t* oid = out_ids + (size_t)(u0 + u) * k;
    float* osc = out_sc ? out_sc + (size_t)(u0 + u) * k : nullptr;
    for (int r = lane; r < k; r += 64) {
        const bool have = r < count;
        oid[r] = have ? L.c.id[r] : -1;
        if (osc) osc[r] = have ? fval(L.c.key[r]) : -INFINITY;
    }
}

// Per user: Recall@k_m or NDCG@k_m (kind 0 / 1) of the ranked list ids[u][0..k) against the held-out
// items hold_idx[hold_ptr[u] .. hold_ptr[u+1]) (ascending); NaN when nothing is held out.
struct MetricSpec {
    int32_t kind[64];
    int32_t k[64];
};

__global__ __launch_bounds__(256) void k_rank_metrics(const int32_t* __restrict__ ids, int64_t n, int32_t k,
                                                      const int64_t* __restrict__ hp, const int32_t* __restrict__ hi,
                                                      int32_t nm, MetricSpec spec, double* __restrict__ out) {
    const int64_t u = blockIdx.x * 256ll + threadIdx.x;
    if (u >= n) return;
    const int64_t lo = hp[u], end = hp[u + 1];
    const int64_t T = end - lo;
    for (int m = 0; m < nm; ++m) {
        const int km = spec.k[m];
        double v = NAN;
        if (T > 0) {
            double hits = 0.0, dcg = 0.0;
            for (int r = 0; r < km; ++r) {
                const int32_t it = ids[u * k + r];
                int64_t a = lo, b = end;  // first position with hold >= it
                while (a < b) {
                    const int64_t c = (a + b) >> 1;
                    if (hi[c] < it) a = c + 1;
                    else b = c;
                }
                if (it >= 0 && a < end && hi[a] == it) {
                    hits += 1.0;
                    dcg += 1.0 / log2((double)r + 2.0);
                }
            }
            const int64_t nideal = std::min<int64_t>(km, T);
            if (spec.kind[m] == 0) {
                v = hits / (double)nideal;
            } else {
                double idcg = 0.0;
                for (int64_t r = 0; r < nideal; ++r) idcg += 1.0 / log2((double)r + 2.0);
                v = dcg / idcg;
            }
        }
        out[u * nm + m] = v;
    }
}

// sums[m] = sum of the non-NaN per-user values of metric m, counts[m] their number; one workgroup,
// each thread takes every 256th user, then a fixed-order tree over the threads.
__global__ __launch_bounds__(256) void k_metric_sums(const double* __restrict__ per_user, int64_t n, int32_t nm,
                                                     double* __restrict__ sums, int64_t* __restrict__ counts) {
    __shared__ double ss[256];
    __shared__ long long cc[256];
    for (int m = 0; m < nm; ++m) {
        double s = 0.0;
        long long c = 0;
        for (int64_t u = threadIdx.x; u < n; u += 256) {
            const double v = per_user[u * nm + m];
            if (v == v) {  // not NaN
                s += v;
                ++c;
            }
        }
        ss[threadIdx.x] = s;
        cc[threadIdx.x] = c;
        __syncthreads();
        for (int h = 128; h > 0; h >>= 1) {
            if ((int)threadIdx.x < h) {
                ss[threadIdx.x] += ss[threadIdx.x + h];
                cc[threadIdx.x] += cc[threadIdx.x + h];
            }
            __syncthreads();
        }
        if (threadIdx.x == 0) {
            sums[m] = ss[0];
            counts[m] = cc[0];
        }
        __syncthreads();
    }
}

bool aligned16(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 15u) == 0; }

// Argument checks shared by both top-k entry points; on success *I4 is n_items rounded up to 4.
ials_status rank_check(const float* W, int64_t n_users, const float* H, int32_t n_items, int32_t d,
                       const int64_t* excl_ptr, const int32_t* excl_idx, int32_t k, const int32_t* out_ids,
                       int32_t* I4) {
    if (n_users < 0 || n_items < 0 || d < 1 || (d & 3) != 0 || k < 1 || k > kMaxK)
        return rank_fail(IALS_E_INVALID, "need n_users >= 0, n_items >= 0, d >= 1 a multiple of 4, 1 <= k <= 512");
    if (n_users == 0) return IALS_OK;
    if (!W || (n_items > 0 && !H) || !out_ids || (excl_ptr == nullptr) != (excl_idx == nullptr))
        return rank_fail(IALS_E_INVALID, "W, H and out_ids must be given; excl_ptr and excl_idx together or neither");
    if (!aligned16(W) || !aligned16(H)) return rank_fail(IALS_E_INVALID, "W and H must be 16-byte aligned");
    if (n_items > INT32_MAX - 4) return rank_fail(IALS_E_INVALID, "too many items");
    *I4 = (n_items + 3) & ~3;
    return IALS_OK;
}

// Scores, exclusions and selection for users [0, n_users) in batches of ub users whose scores
// fit S (ub * I4 floats).
void rank_batches(const float* W, int64_t n_users, const float* H, int32_t n_items, int32_t d, int32_t I4,
                  const int64_t* excl_ptr, const int32_t* excl_idx, int32_t k, int32_t* out_ids, float* out_scores,
                  float* S, int64_t ub, hipStream_t st) {
    for (int64_t u0 = 0; u0 < n_users; u0 += ub) {
        const int32_t nu = (int32_t)std::min<int64_t>(ub, n_users - u0);
        if (I4 > 0) {
            const int64_t n_it = (I4 + 127) / 128, ipx = (n_it + 7) / 8, n_ut = (nu + 127) / 128;
            hipLaunchKernelGGL(k_score, dim3((unsigned)(8 * ipx * n_ut)), dim3(256), 0, st, W, H, d, u0, nu, n_items,
                               I4, S);
            if (excl_ptr)
                hipLaunchKernelGGL(k_mask_excl, dim3((unsigned)((nu + 3) / 4)), dim3(256), 0, st, excl_ptr, excl_idx, u0,
                                   nu, n_items, I4, S);
        }
        hipLaunchKernelGGL(k_select, dim3((unsigned)((nu + 3) / 4)), dim3(256), 0, st, S, nu, I4, k, u0, out_ids,
                           out_scores);
    }
}

// Device address of `scratch` on the current device, looked up once per device.
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
float* g_scratch_ptr[kMaxDevices] = {};

ials_status scratch_on_current_device(float** out) {
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return rank_fail(IALS_E_HIP, std::string("hipGetDevice failed: ") + hipGetErrorString(e));
    if (dev < 0 || dev >= kMaxDevices) return rank_fail(IALS_E_INVALID, "device index beyond the supported 64");
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return rank_fail(IALS_E_HIP, std::string("hipGetSymbolAddress of the score scratch failed: ") +
                                             hipGetErrorString(e));
        g_scratch_ptr[dev] = static_cast<float*>(p);
    }
    *out = g_scratch_ptr[dev];
    return IALS_OK;
}

}  // namespace

extern "C" {

ials_status ials_rank_topk(const float* W, int64_t n_users, const float* H, int32_t n_items, int32_t d,
                           const int64_t* excl_ptr, const int32_t* excl_idx, int32_t k, int32_t* out_ids,
                           float* out_scores, int64_t score_buffer_bytes, void* stream) {
    int32_t I4 = 0;
    ials_status s = rank_check(W, n_users, H, n_items, d, excl_ptr, excl_idx, k, out_ids, &I4);
    if (s != IALS_OK || n_users == 0) return s;
    hipStream_t st = (hipStream_t)stream;
    if (score_buffer_bytes <= 0) score_buffer_bytes = int64_t(1) << 30;
    const int64_t row_bytes = std::max<int64_t>(16, (int64_t)I4 * 4);
    const int64_t ub = std::max<int64_t>(1, std::min<int64_t>(n_users, score_buffer_bytes / row_bytes));
    if (ub * (int64_t)I4 > (int64_t(1) << 40)) return rank_fail(IALS_E_INVALID, "score buffer too large");
    float* S = nullptr;
    if (I4 > 0) {
        if (hipMallocAsync((void**)&S, (size_t)(ub * I4) * sizeof(float), st) != hipSuccess) {
            (void)hipGetLastError();
            return rank_fail(IALS_E_NOMEM, "score buffer allocation failed");
        }
    }
    rank_batches(W, n_users, H, n_items, d, I4, excl_ptr, excl_idx, k, out_ids, out_scores, S, ub, st);
    if (S) (void)hipFreeAsync(S, st);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return rank_fail(IALS_E_HIP, std::string("launch failed: ") + hipGetErrorString(e));
    return IALS_OK;
}

ials_status ials_rank_topk_noalloc(const float* W, int64_t n_users, const float* H, int32_t n_items, int32_t d,
                                   const int64_t* excl_ptr, const int32_t* excl_idx, int32_t k, int32_t* out_ids,
                                   float* out_scores, void* stream) {
    int32_t I4 = 0;
    ials_status s = rank_check(W, n_users, H, n_items, d, excl_ptr, excl_idx, k, out_ids, &I4);
    if (s != IALS_OK || n_users == 0) return s;
    const int64_t row_bytes = std::max<int64_t>(16, (int64_t)I4 * 4);
    if (row_bytes > (int64_t)kRankScratchBytes)
        return rank_fail(IALS_E_INVALID, "one user's scores need " + std::to_string(row_bytes) +
                                             " bytes, more than the fixed score scratch of " +
                                             std::to_string(kRankScratchBytes) + " bytes (n_items <= " +
                                             std::to_string(kRankScratchBytes / 4) + ")");
    float* S = nullptr;
    s = scratch_on_current_device(&S);
    if (s != IALS_OK) return s;
    const int64_t ub = std::min<int64_t>(n_users, (int64_t)kRankScratchBytes / row_bytes);
    rank_batches(W, n_users, H, n_items, d, I4, excl_ptr, excl_idx, k, out_ids, out_scores, S, ub,
                 (hipStream_t)stream);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return rank_fail(IALS_E_HIP, std::string("launch failed: ") + hipGetErrorString(e));
    return IALS_OK;
}

ials_status ials_rank_metrics(const int32_t* ids, int64_t n_users, int32_t k, const int64_t* hold_ptr,
                              const int32_t* hold_idx, int32_t n_metrics, const int32_t* kinds, const int32_t* ks,
                              double* per_user, double* sums_host, int64_t* counts_host, void* stream) {
    if (n_users < 0 || k < 1 || n_metrics < 1 || n_metrics > 64 || !kinds || !ks || !sums_host || !counts_host)
        return rank_fail(IALS_E_INVALID, "need n_users >= 0, k >= 1, 1 <= n_metrics <= 64 and host kinds/ks/sums/counts");
    for (int m = 0; m < n_metrics; ++m)
        if ((kinds[m] != 0 && kinds[m] != 1) || ks[m] < 1 || ks[m] > k)
            return rank_fail(IALS_E_INVALID, "metric kinds are 0 (recall) or 1 (ndcg), with 1 <= k_m <= k");
    if (n_users > 0 && (!ids || !hold_ptr || !hold_idx || !per_user))
        return rank_fail(IALS_E_INVALID, "ids, hold_ptr, hold_idx and per_user must be given");
    hipStream_t st = (hipStream_t)stream;
    for (int m = 0; m < n_metrics; ++m) {
        sums_host[m] = 0.0;
        counts_host[m] = 0;
    }
    if (n_users == 0) return IALS_OK;
    MetricSpec spec{};
    for (int m = 0; m < n_metrics; ++m) {
        spec.kind[m] = kinds[m];
        spec.k[m] = ks[m];
    }
    double* dsum = nullptr;  // [64] sums, then [64] counts
    if (hipMallocAsync((void**)&dsum, sizeof(double) * 64 + sizeof(int64_t) * 64, st) != hipSuccess) {
        (void)hipGetLastError();
        return rank_fail(IALS_E_NOMEM, "metric scratch allocation failed");
    }
    int64_t* dcnt = reinterpret_cast<int64_t*>(dsum + 64);
    hipLaunchKernelGGL(k_rank_metrics, dim3((unsigned)((n_users + 255) / 256)), dim3(256), 0, st, ids, n_users, k,
                       hold_ptr, hold_idx, n_metrics, spec, per_user);
    hipLaunchKernelGGL(k_metric_sums, dim3(1), dim3(256), 0, st, per_user, n_users, n_metrics, dsum, dcnt);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) e = hipMemcpyAsync(sums_host, dsum, sizeof(double) * n_metrics, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipMemcpyAsync(counts_host, dcnt, sizeof(int64_t) * n_metrics, hipMemcpyDeviceToHost, st);
    (void)hipFreeAsync(dsum, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return rank_fail(IALS_E_HIP, std::string("metrics failed: ") + hipGetErrorString(e));
    return IALS_OK;
}

const char* ials_rank_last_error(void) { return g_rank_error.c_str(); }

}  // extern "C"
