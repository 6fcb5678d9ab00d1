// Stable LSD radix sort of (key, value) pairs, 4 bits per pass.
//
// Used where particles arrive in arbitrary order: encoding float input into
// the cell-ordered state (Sec. III-A, stable with respect to the input order)
// and the fallback compaction when a particle moves more than one coarse cell
// in a step.  Each pass: per-tile digit histograms, one exclusive scan over
// the digit-major histogram, then a stable scatter whose in-tile ranks come
// from wavefront ballots.
#include "common.h"

namespace cube {

namespace {

constexpr int kSortThreads = 256;
constexpr int kSortItems = 16;
constexpr int kSortTile = kSortThreads * kSortItems;
constexpr int kRadixBits = 4;
constexpr int kRadix = 1 << kRadixBits;
constexpr int kSortWaves = kSortThreads / kWave;

__global__ __launch_bounds__(kSortThreads) void k_digit_hist(const uint32_t* __restrict__ key, int64_t n,
                                                              int shift, int64_t nb,
                                                              int32_t* __restrict__ hist) {
    __shared__ int cnt[kRadix];
    if (threadIdx.x < kRadix) cnt[threadIdx.x] = 0;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * kSortTile;
    int local[kRadix];
#pragma unroll
    for (int d = 0; d < kRadix; ++d) local[d] = 0;
#pragma unroll
    for (int it = 0; it < kSortItems; ++it) {
        int64_t e = base + it * kSortThreads + threadIdx.x;
        if (e < n) {
            int d = (key[e] >> shift) & (kRadix - 1);
#pragma unroll
            for (int q = 0; q < kRadix; ++q) local[q] += (d == q);
        }
    }
#pragma unroll
    for (int d = 0; d < kRadix; ++d) {
        int v = wave_sum(local[d]);
        if ((threadIdx.x & (kWave - 1)) == 0 && v) atomicAdd(&cnt[d], v);
    }
    __syncthreads();
    if (threadIdx.x < kRadix) hist[(int64_t)threadIdx.x * nb + blockIdx.x] = cnt[threadIdx.x];
}

__global__ __launch_bounds__(kSortThreads) void k_digit_scatter(
    const uint32_t* __restrict__ key, const uint32_t* __restrict__ val, int64_t n, int shift, int64_t nb,
    const int32_t* __restrict__ base_of, uint32_t* __restrict__ key_out, uint32_t* __restrict__ val_out) {
    __shared__ int wc[kSortItems][kSortWaves][kRadix];
    const int lane = threadIdx.x & (kWave - 1);
    const int wid = threadIdx.x / kWave;
    const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (kWave - lane));
    const int64_t base = (int64_t)blockIdx.x * kSortTile;
    uint32_t k[kSortItems], v[kSortItems];
    int dig[kSortItems], rank[kSortItems];
#pragma unroll
    for (int it = 0; it < kSortItems; ++it) {
        int64_t e = base + it * kSortThreads + threadIdx.x;
        const bool ok = e < n;
        k[it] = ok ? key[e] : 0u;
        v[it] = ok ? val[e] : 0u;
        dig[it] = ok ? (int)((k[it] >> shift) & (kRadix - 1)) : kRadix;
        uint64_t mine = 0;
#pragma unroll
        for (int d = 0; d < kRadix; ++d) {
            uint64_t m = __ballot(dig[it] == d);
            if (lane == d) wc[it][wid][d] = __popcll(m);
            if (dig[it] == d) mine = m;
        }
        rank[it] = __popcll(mine & lt);
    }
    __syncthreads();
    // exclusive prefix per digit in (item, wave) order, plus the global base
    if (threadIdx.x < kRadix) {
        const int d = threadIdx.x;
        int acc = base_of[(int64_t)d * nb + blockIdx.x];
        for (int it = 0; it < kSortItems; ++it)
            for (int w = 0; w < kSortWaves; ++w) {
                int t = wc[it][w][d];
                wc[it][w][d] = acc;
                acc += t;
            }
    }
    __syncthreads();
#pragma unroll
    for (int it = 0; it < kSortItems; ++it) {
        if (dig[it] < kRadix) {
            int64_t o = (int64_t)wc[it][wid][dig[it]] + rank[it];
            key_out[o] = k[it];
            val_out[o] = v[it];
        }
    }
}

}  // namespace

size_t sort_workspace_bytes(int64_t n) {
    int64_t nb = (n + kSortTile - 1) / kSortTile;
    int64_t h = (int64_t)kRadix * nb;
    return (size_t)(2 * ((h + 1 + 15) / 16 * 16)) * sizeof(int32_t) + scan_workspace_bytes(h) + 256;
}

void stable_sort_pairs(uint32_t* key, uint32_t* val, uint32_t* key_tmp, uint32_t* val_tmp,
                       int64_t n, int bits, void* ws, hipStream_t s) {
    if (n <= 1 || bits <= 0) return;
    const int64_t nb = (n + kSortTile - 1) / kSortTile;
    const int64_t h = (int64_t)kRadix * nb;
    int32_t* hist = static_cast<int32_t*>(ws);
    int32_t* hscan = hist + (h + 1 + 15) / 16 * 16;
    void* scan_ws = hscan + (h + 1 + 15) / 16 * 16;
    uint32_t *ki = key, *vi = val, *ko = key_tmp, *vo = val_tmp;
    int passes = 0;
    for (int shift = 0; shift < bits; shift += kRadixBits, ++passes) {
        hipLaunchKernelGGL(k_digit_hist, dim3((unsigned)nb), dim3(kSortThreads), 0, s, ki, n, shift, nb, hist);
        exclusive_scan_i32(hist, hscan, h, scan_ws, s);
        hipLaunchKernelGGL(k_digit_scatter, dim3((unsigned)nb), dim3(kSortThreads), 0, s, ki, vi, n, shift,
                           nb, hscan, ko, vo);
        uint32_t* t = ki; ki = ko; ko = t;
        t = vi; vi = vo; vo = t;
    }
    if (passes & 1) {
        hipMemcpyAsync(key, ki, n * sizeof(uint32_t), hipMemcpyDeviceToDevice, s);
        hipMemcpyAsync(val, vi, n * sizeof(uint32_t), hipMemcpyDeviceToDevice, s);
    }
}

}  // namespace cube
