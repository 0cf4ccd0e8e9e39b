// Observation index on the device: user-major CSR (the yhat order), item-major
// CSR with the permutation back to user-major slots, row schedules by length and
// the segment table of long rows.  The per-user and per-item loops of Alg. 3
// ("for (u*, i, y, alpha) in S") walk these segments.
//
// Both orders come from a stable LSD radix sort of 64-bit keys (row * ncols + col)
// written for wave64: 8-bit digits, per-tile histograms, a device scan, and a
// stable scatter that ranks equal digits inside a wavefront with ballots.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <vector>

#include "ials_internal.h"

namespace ials {
namespace {

constexpr int kRsThreads = 256;
constexpr int kRsItems = 16;
constexpr int kRsTile = kRsThreads * kRsItems;
constexpr int kScanThreads = 256;
constexpr int kScanItems = 8;
constexpr int kScanTile = kScanThreads * kScanItems;

__global__ void k_rs_hist(const uint64_t* __restrict__ keys, int64_t n, int shift,
                          uint32_t* __restrict__ hist, int64_t nblocks) {
    __shared__ uint32_t cnt[256];
    cnt[threadIdx.x] = 0;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * kRsTile;
    for (int j = 0; j < kRsItems; ++j) {
        int64_t e = base + (int64_t)j * kRsThreads + threadIdx.x;
        if (e < n) atomicAdd(&cnt[(keys[e] >> shift) & 255u], 1u);
    }
    __syncthreads();
    hist[(int64_t)threadIdx.x * nblocks + blockIdx.x] = cnt[threadIdx.x];
}

// Exclusive scan, phase 1: each block scans kScanTile elements in place and
// records its total.
template <typename T>
__global__ void k_scan_tile(T* __restrict__ v, int64_t n, T* __restrict__ sums) {
    __shared__ T part[kScanThreads];
    const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
    T loc[kScanItems];
    T s = 0;
    for (int j = 0; j < kScanItems; ++j) {
        int64_t e = base + j;
        loc[j] = (e < n) ? v[e] : T(0);
        s += loc[j];
    }
    part[threadIdx.x] = s;
    __syncthreads();
    // Hillis-Steele inclusive scan over the thread totals.
    for (int off = 1; off < kScanThreads; off <<= 1) {
        T t = (threadIdx.x >= (unsigned)off) ? part[threadIdx.x - off] : T(0);
        __syncthreads();
        part[threadIdx.x] += t;
        __syncthreads();
    }
    T run = (threadIdx.x > 0) ? part[threadIdx.x - 1] : T(0);
    for (int j = 0; j < kScanItems; ++j) {
        int64_t e = base + j;
        if (e < n) v[e] = run;
        run += loc[j];
    }
    if (threadIdx.x == kScanThreads - 1) sums[blockIdx.x] = part[kScanThreads - 1];
}

// Phase 2: exclusive scan of the block totals by one block (serial chunks).
template <typename T>
__global__ void k_scan_sums(T* __restrict__ sums, int64_t nb) {
    __shared__ T part[kScanThreads];
    __shared__ T carry;
    if (threadIdx.x == 0) carry = 0;
    __syncthreads();
    for (int64_t c0 = 0; c0 < nb; c0 += kScanThreads) {
        int64_t e = c0 + threadIdx.x;
        T x = (e < nb) ? sums[e] : T(0);
        part[threadIdx.x] = x;
        __syncthreads();
        for (int off = 1; off < kScanThreads; off <<= 1) {
            T t = (threadIdx.x >= (unsigned)off) ? part[threadIdx.x - off] : T(0);
            __syncthreads();
            part[threadIdx.x] += t;
            __syncthreads();
        }
        if (e < nb) sums[e] = carry + part[threadIdx.x] - x;
        __syncthreads();
        if (threadIdx.x == 0) carry += part[kScanThreads - 1];
        __syncthreads();
    }
}

template <typename T>
__global__ void k_scan_add(T* __restrict__ v, int64_t n, const T* __restrict__ sums) {
    const int64_t base = (int64_t)blockIdx.x * kScanTile;
    const T add = sums[blockIdx.x];
    for (int j = threadIdx.x; j < kScanTile; j += kScanThreads) {
        int64_t e = base + j;
        if (e < n) v[e] += add;
    }
}

// Stable scatter of one digit pass.  Keys of a tile are visited round by round
// (kRsThreads consecutive keys per round, in index order); inside a round a
// wavefront ranks equal digits with ballots, and waves are ordered by index.
__global__ __launch_bounds__(kRsThreads) void k_rs_scatter(const uint64_t* __restrict__ kin,
                                                           const int32_t* __restrict__ vin,
                                                           uint64_t* __restrict__ kout,
                                                           int32_t* __restrict__ vout, int64_t n, int shift,
                                                           const uint32_t* __restrict__ offs, int64_t nblocks) {
    constexpr int kWaves = kRsThreads / kWave;
    __shared__ uint32_t base[256];
    __shared__ uint32_t wcnt[kWaves][256];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    base[tid] = offs[(int64_t)tid * nblocks + blockIdx.x];
    const uint64_t lt_mask = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    const int64_t tile = (int64_t)blockIdx.x * kRsTile;
    for (int j = 0; j < kRsItems; ++j) {
        for (int w = 0; w < kWaves; ++w) wcnt[w][tid] = 0;
        __syncthreads();
        const int64_t e = tile + (int64_t)j * kRsThreads + tid;
        const bool valid = e < n;
        uint64_t key = valid ? kin[e] : 0;
        int32_t val = valid ? vin[e] : 0;
        const uint32_t dig = (uint32_t)((key >> shift) & 255u);
        uint64_t peers = __ballot(valid);
        for (int bit = 0; bit < 8; ++bit) {
            const bool on = (dig >> bit) & 1u;
            const uint64_t m = __ballot(on);
            peers &= on ? m : ~m;
        }
        const uint32_t rank = (uint32_t)__popcll(peers & lt_mask);
        if (valid && rank == 0) wcnt[wave][dig] = (uint32_t)__popcll(peers);
        __syncthreads();
        if (valid) {
            uint32_t before = 0;
            for (int w = 0; w < wave; ++w) before += wcnt[w][dig];
            const uint32_t dst = base[dig] + before + rank;
            kout[dst] = key;
            vout[dst] = val;
        }
        __syncthreads();
        uint32_t tot = 0;
        for (int w = 0; w < kWaves; ++w) tot += wcnt[w][tid];
        base[tid] += tot;
        __syncthreads();
    }
}

__global__ void k_validate(const int32_t* __restrict__ u, const int32_t* __restrict__ i, int64_t n, int32_t U,
                           int32_t I, const float* __restrict__ a, unsigned long long* counters) {
    int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    bool bad = u[k] < 0 || u[k] >= U || i[k] < 0 || i[k] >= I;
    if (a && !(a[k] > 0.f)) bad = true;
    if (bad) atomicAdd(&counters[CNT_BAD_INPUT], 1ull);
}

__global__ void k_make_keys(const int32_t* __restrict__ row, const int32_t* __restrict__ col, int64_t n,
                            int64_t ncols, uint64_t* __restrict__ keys, int32_t* __restrict__ vals) {
    int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    keys[k] = (uint64_t)row[k] * (uint64_t)ncols + (uint64_t)col[k];
    vals[k] = (int32_t)k;
}

// After the user-major sort: col, row-boundaries, duplicate check, and the keys
// of the item-major sort (item * U + user) with the user slot as value.
__global__ void k_user_side(const uint64_t* __restrict__ keys, int64_t n, int64_t I, int64_t U,
                            int32_t* __restrict__ ucol, int64_t* __restrict__ uptr, uint64_t* __restrict__ ikeys,
                            int32_t* __restrict__ ivals, unsigned long long* counters) {
    int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n) return;
    const uint64_t k = keys[s];
    const int64_t r = (int64_t)(k / (uint64_t)I), c = (int64_t)(k % (uint64_t)I);
    ucol[s] = (int32_t)c;
    ikeys[s] = (uint64_t)c * (uint64_t)U + (uint64_t)r;
    ivals[s] = (int32_t)s;
    const int64_t rprev = (s == 0) ? -1 : (int64_t)(keys[s - 1] / (uint64_t)I);
    if (s > 0 && keys[s - 1] == k) atomicAdd(&counters[CNT_DUPLICATE], 1ull);
    for (int64_t rr = rprev + 1; rr <= r; ++rr) uptr[rr] = s;
    if (s == n - 1)
        for (int64_t rr = r + 1; rr <= U; ++rr) uptr[rr] = n;
}

__global__ void k_item_side(const uint64_t* __restrict__ keys, int64_t n, int64_t U, int64_t I,
                            int32_t* __restrict__ icol, int64_t* __restrict__ iptr) {
    int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n) return;
    const uint64_t k = keys[s];
    const int64_t r = (int64_t)(k / (uint64_t)U), c = (int64_t)(k % (uint64_t)U);
    icol[s] = (int32_t)c;
    const int64_t rprev = (s == 0) ? -1 : (int64_t)(keys[s - 1] / (uint64_t)U);
    for (int64_t rr = rprev + 1; rr <= r; ++rr) iptr[rr] = s;
    if (s == n - 1)
        for (int64_t rr = r + 1; rr <= I; ++rr) iptr[rr] = n;
}

__global__ void k_fill_i64(int64_t* p, int64_t n, int64_t v) {
    int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k < n) p[k] = v;
}

template <typename T>
__global__ void k_gather(const T* __restrict__ src, const int32_t* __restrict__ idx, int64_t n, T* __restrict__ dst) {
    int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k < n) dst[k] = src[idx[k]];
}

// Keys for ordering rows by decreasing length (stable: equal lengths keep row order).
__global__ void k_len_keys(const int64_t* __restrict__ ptr, int32_t nrows, int32_t seg_len,
                           uint64_t* __restrict__ keys, int32_t* __restrict__ vals, int32_t* __restrict__ nseg) {
    int32_t r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= nrows) return;
    const int64_t len = ptr[r + 1] - ptr[r];
    keys[r] = 0xFFFFFFFFull - (uint64_t)len;
    vals[r] = r;
    nseg[r] = (len > seg_len) ? (int32_t)((len + seg_len - 1) / seg_len) : 0;
}

// Sort key of each segment: its first partner id (then the segment id, for a total order).
__global__ void k_seg_keys(const int64_t* __restrict__ seg_lo, const int32_t* __restrict__ col, int32_t nseg,
                           uint64_t* __restrict__ keys, int32_t* __restrict__ vals) {
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= nseg) return;
    keys[s] = ((uint64_t)(uint32_t)col[seg_lo[s]] << 32) | (uint32_t)s;
    vals[s] = s;
}

__global__ void k_seg_fill(const int64_t* __restrict__ ptr, int32_t nrows, int32_t seg_len,
                           const int32_t* __restrict__ nseg_scan,
                           const int32_t* __restrict__ nseg, int32_t* __restrict__ seg_first,
                           int32_t* __restrict__ seg_row, int64_t* __restrict__ seg_lo, int64_t* __restrict__ seg_hi) {
    int32_t r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= nrows) return;
    const int32_t cnt = nseg[r];
    if (cnt == 0) {
        seg_first[r] = -1;
        return;
    }
    const int32_t f = nseg_scan[r];
    seg_first[r] = f;
    const int64_t lo = ptr[r], hi = ptr[r + 1];
    for (int32_t j = 0; j < cnt; ++j) {
        seg_row[f + j] = r;
        seg_lo[f + j] = lo + (int64_t)j * seg_len;
        seg_hi[f + j] = std::min(hi, lo + (int64_t)(j + 1) * seg_len);
    }
}

inline unsigned nblk(int64_t n, int t) { return (unsigned)((n + t - 1) / t); }

template <typename T>
hipError_t scan_exclusive(T* v, int64_t n, T* tmp_sums, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    const int64_t nb = (n + kScanTile - 1) / kScanTile;
    hipLaunchKernelGGL(k_scan_tile<T>, dim3((unsigned)nb), dim3(kScanThreads), 0, st, v, n, tmp_sums);
    hipLaunchKernelGGL(k_scan_sums<T>, dim3(1), dim3(kScanThreads), 0, st, tmp_sums, nb);
    hipLaunchKernelGGL(k_scan_add<T>, dim3((unsigned)nb), dim3(kScanThreads), 0, st, v, n, tmp_sums);
    return hipGetLastError();
}

int bits_for(uint64_t maxkey) {
    int b = 0;
    while (b < 64 && (maxkey >> b) != 0) ++b;
    return b;
}

// Sort (keys, vals) of length n; keys < 2^nbits.  Result in (keys, vals).
hipError_t radix_sort(uint64_t* keys, int32_t* vals, uint64_t* kalt, int32_t* valt, int64_t n, int nbits,
                      uint32_t* hist, uint32_t* sums, hipStream_t st) {
    if (n <= 1) return hipSuccess;
    const int64_t nb = (n + kRsTile - 1) / kRsTile;
    uint64_t *ki = keys, *ko = kalt;
    int32_t *vi = vals, *vo = valt;
    const int passes = (nbits + 7) / 8;
    for (int p = 0; p < passes; ++p) {
        const int shift = 8 * p;
        hipLaunchKernelGGL(k_rs_hist, dim3((unsigned)nb), dim3(kRsThreads), 0, st, ki, n, shift, hist, nb);
        hipError_t e = scan_exclusive<uint32_t>(hist, 256 * nb, sums, st);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(k_rs_scatter, dim3((unsigned)nb), dim3(kRsThreads), 0, st, ki, vi, ko, vo, n, shift,
                           hist, nb);
        std::swap(ki, ko);
        std::swap(vi, vo);
    }
    if (ki != keys) {
        hipError_t e = hipMemcpyAsync(keys, ki, sizeof(uint64_t) * n, hipMemcpyDeviceToDevice, st);
        if (e != hipSuccess) return e;
        e = hipMemcpyAsync(vals, vi, sizeof(int32_t) * n, hipMemcpyDeviceToDevice, st);
        if (e != hipSuccess) return e;
    }
    return hipGetLastError();
}

// Temporaries of the index build, counted against the context's budget while held.
struct TmpBuf {
    ials_ctx* c;
    std::vector<std::pair<void*, size_t>> ptrs;
    explicit TmpBuf(ials_ctx* ctx) : c(ctx) {}
    ~TmpBuf() {
        (void)hipStreamSynchronize(c->stream);
        for (auto& pb : ptrs) tmp_free(c, pb.first, pb.second);
    }
    template <typename T>
    hipError_t get(T** p, size_t count) {
        void* q = nullptr;
        const size_t bytes = std::max<size_t>(count, 1) * sizeof(T);
        hipError_t e = tmp_alloc(c, &q, bytes);
        if (e == hipSuccess) ptrs.emplace_back(q, bytes);
        *p = (T*)q;
        return e;
    }
};

}  // namespace

// Build both observation indices, the per-side label arrays, row orders and
// segment tables.  d_user/d_item/d_y/d_a are device arrays in the caller's order.
ials_status build_index(ials_ctx* c, const int32_t* d_user, const int32_t* d_item, const float* d_y,
                        const float* d_a) {
    hipStream_t st = c->stream;
    const int64_t n = c->nnz;
    const int64_t U = c->U, I = c->I;
    TmpBuf tmp(c);
    uint64_t *keys, *kalt;
    int32_t *vals, *valt;
    uint32_t *hist, *sums;
    const int64_t nmax = std::max<int64_t>({n, U, I, 1});
    const int64_t nbmax = (nmax + kRsTile - 1) / kRsTile;
    IALS_ALLOC_TRY(c, tmp.get(&keys, nmax));
    IALS_ALLOC_TRY(c, tmp.get(&kalt, nmax));
    IALS_ALLOC_TRY(c, tmp.get(&vals, nmax));
    IALS_ALLOC_TRY(c, tmp.get(&valt, nmax));
    IALS_ALLOC_TRY(c, tmp.get(&hist, 256 * nbmax));
    IALS_ALLOC_TRY(c, tmp.get(&sums, (256 * nbmax + nmax + 2) / kScanTile + 2));

    // validation of ids and weights, before any index is derived from them
    if (n > 0) {
        hipLaunchKernelGGL(k_validate, dim3(nblk(n, 256)), dim3(256), 0, st, d_user, d_item, n, c->U, c->I, d_a,
                           c->counters);
        long long bad = 0;
        IALS_HIP_TRY(c, hipMemcpyAsync(&bad, c->counters + CNT_BAD_INPUT, sizeof(bad), hipMemcpyDeviceToHost, st));
        IALS_HIP_TRY(c, hipStreamSynchronize(st));
        if (bad != 0) {
            c->err = std::to_string(bad) + " observations have an id out of range or a weight <= 0";
            return IALS_E_INVALID;
        }
    }
    // user-major order
    SideIndex& us = c->side[IALS_SIDE_USER];
    SideIndex& is = c->side[IALS_SIDE_ITEM];
    if (n > 0) {
        hipLaunchKernelGGL(k_make_keys, dim3(nblk(n, 256)), dim3(256), 0, st, d_user, d_item, n, I, keys, vals);
        IALS_HIP_TRY(c, radix_sort(keys, vals, kalt, valt, n, bits_for((uint64_t)U * I - 1), hist, sums, st));
        // vals = source index of every user slot; keys = user*I + item.
        // kalt/valt become the item-major keys (item*U + user) and user slots.
        hipLaunchKernelGGL(k_user_side, dim3(nblk(n, 256)), dim3(256), 0, st, keys, n, I, U, us.col, us.ptr, kalt,
                           valt, c->counters);
        long long dup = 0;
        IALS_HIP_TRY(c, hipMemcpyAsync(&dup, c->counters + CNT_DUPLICATE, sizeof(dup), hipMemcpyDeviceToHost, st));
        IALS_HIP_TRY(c, hipStreamSynchronize(st));
        if (dup != 0) {
            c->err = std::to_string(dup) + " repeated (user, item) pairs";
            return IALS_E_INVALID;
        }
        if (d_y && us.y) hipLaunchKernelGGL(k_gather<float>, dim3(nblk(n, 256)), dim3(256), 0, st, d_y, vals, n, us.y);
        if (d_a && us.a) hipLaunchKernelGGL(k_gather<float>, dim3(nblk(n, 256)), dim3(256), 0, st, d_a, vals, n, us.a);
        // item-major order: sort (item*U + user, user slot)
        IALS_HIP_TRY(c, radix_sort(kalt, valt, keys, vals, n, bits_for((uint64_t)I * U - 1), hist, sums, st));
        hipLaunchKernelGGL(k_item_side, dim3(nblk(n, 256)), dim3(256), 0, st, kalt, n, U, I, is.col, is.ptr);
        IALS_HIP_TRY(c, hipMemcpyAsync(is.slot, valt, sizeof(int32_t) * n, hipMemcpyDeviceToDevice, st));
        if (us.y && is.y) hipLaunchKernelGGL(k_gather<float>, dim3(nblk(n, 256)), dim3(256), 0, st, us.y, is.slot, n, is.y);
        if (us.a && is.a) hipLaunchKernelGGL(k_gather<float>, dim3(nblk(n, 256)), dim3(256), 0, st, us.a, is.slot, n, is.a);
    } else {
        hipLaunchKernelGGL(k_fill_i64, dim3(nblk(U + 1, 256)), dim3(256), 0, st, us.ptr, U + 1, (int64_t)0);
        hipLaunchKernelGGL(k_fill_i64, dim3(nblk(I + 1, 256)), dim3(256), 0, st, is.ptr, I + 1, (int64_t)0);
    }
    IALS_HIP_TRY(c, hipGetLastError());

    // row orders and segment tables
    for (int sd = 0; sd < 2; ++sd) {
        SideIndex& s = c->side[sd];
        const int32_t nr = s.nrows;
        int32_t* nseg;
        IALS_ALLOC_TRY(c, tmp.get(&nseg, nr + 1));
        hipLaunchKernelGGL(k_len_keys, dim3(nblk(nr, 256)), dim3(256), 0, st, s.ptr, nr, c->seg_len, keys, vals, nseg);
        IALS_HIP_TRY(c, radix_sort(keys, vals, kalt, valt, nr, 32, hist, sums, st));
        IALS_HIP_TRY(c, hipMemcpyAsync(s.order, vals, sizeof(int32_t) * nr, hipMemcpyDeviceToDevice, st));
        // longest row length (first in the order)
        uint64_t k0 = 0xFFFFFFFFull;
        if (nr > 0) IALS_HIP_TRY(c, hipMemcpyAsync(&k0, keys, sizeof(uint64_t), hipMemcpyDeviceToHost, st));
        int32_t* scan;
        IALS_ALLOC_TRY(c, tmp.get(&scan, nr + 1));
        IALS_HIP_TRY(c, hipMemcpyAsync(scan, nseg, sizeof(int32_t) * nr, hipMemcpyDeviceToDevice, st));
        IALS_HIP_TRY(c, hipMemsetAsync(scan + nr, 0, sizeof(int32_t), st));
        IALS_HIP_TRY(c, scan_exclusive<int32_t>(scan, nr + 1, (int32_t*)sums, st));
        int32_t total = 0;
        IALS_HIP_TRY(c, hipMemcpyAsync(&total, scan + nr, sizeof(int32_t), hipMemcpyDeviceToHost, st));
        IALS_HIP_TRY(c, hipStreamSynchronize(st));
        s.max_len = (int64_t)(0xFFFFFFFFull - k0);
        if (nr == 0) s.max_len = 0;
        s.nseg = total;
        if (total > 0) {
            IALS_ALLOC_TRY(c, dev_alloc(c, (void**)&s.seg_row, sizeof(int32_t) * total));
            IALS_ALLOC_TRY(c, dev_alloc(c, (void**)&s.seg_lo, sizeof(int64_t) * total));
            IALS_ALLOC_TRY(c, dev_alloc(c, (void**)&s.seg_hi, sizeof(int64_t) * total));
        }
        hipLaunchKernelGGL(k_seg_fill, dim3(nblk(nr, 256)), dim3(256), 0, st, s.ptr, nr, c->seg_len, scan, nseg, s.seg_first,
                           s.seg_row, s.seg_lo, s.seg_hi);
        IALS_HIP_TRY(c, hipGetLastError());
        // processing order of the segments: by first partner id, so that the segments in flight
        // at one time gather from neighbouring partner rows (long rows' segments are narrow id
        // ranges) and share the L2
        if (total > 0) {
            IALS_ALLOC_TRY(c, dev_alloc(c, (void**)&s.seg_order, sizeof(int32_t) * total));
            hipLaunchKernelGGL(k_seg_keys, dim3(nblk(total, 256)), dim3(256), 0, st, s.seg_lo, s.col, total, keys, vals);
            IALS_HIP_TRY(c, radix_sort(keys, vals, kalt, valt, total, 64, hist, sums, st));
            IALS_HIP_TRY(c, hipMemcpyAsync(s.seg_order, vals, sizeof(int32_t) * total, hipMemcpyDeviceToDevice, st));
        }
        // number of long rows
        if (nr > 0) {
            std::vector<int32_t> h_nseg(nr);
            IALS_HIP_TRY(c, hipMemcpyAsync(h_nseg.data(), nseg, sizeof(int32_t) * nr, hipMemcpyDeviceToHost, st));
            IALS_HIP_TRY(c, hipStreamSynchronize(st));
            s.nlong = (int32_t)std::count_if(h_nseg.begin(), h_nseg.end(), [](int32_t v) { return v > 0; });
        }
    }
    IALS_HIP_TRY(c, hipStreamSynchronize(st));
    return IALS_OK;
}

}  // namespace ials
