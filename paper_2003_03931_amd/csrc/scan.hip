// Exclusive prefix sum of int32 cell counts -> cell offsets (Sec. III-A: a
// per-cell count locates each cell's particles in the cell-ordered arrays).
//
// Three passes over tiles of 4096 values: per-tile totals, a (recursive) scan
// of the totals, then a tile-local scan plus the tile's base.  Each thread
// owns 16 consecutive values so the loads are 64-byte vectors.
#include <algorithm>

#include "common.h"

namespace cube {

namespace {

constexpr int kScanThreads = 256;
constexpr int kScanItems = 16;
constexpr int kScanTile = kScanThreads * kScanItems;

__device__ __forceinline__ bool gated(const int32_t* gate) { return gate && *(volatile const int32_t*)gate; }

__global__ __launch_bounds__(kScanThreads) void k_tile_sums(const int32_t* __restrict__ in,
                                                             int64_t n, int32_t* __restrict__ sums,
                                                             int32_t* __restrict__ max_out, const int32_t* gate) {
    if (gated(gate)) return;
    __shared__ int lds[kScanThreads / kWave + 1];
    const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
    int acc = 0, mx = 0;
    if (base + kScanItems <= n) {
        const int4* p = reinterpret_cast<const int4*>(in + base);
#pragma unroll
        for (int i = 0; i < kScanItems / 4; ++i) {
            int4 q = p[i];
            acc += q.x + q.y + q.z + q.w;
            mx = max(max(mx, max(q.x, q.y)), max(q.z, q.w));
        }
    } else {
        for (int i = 0; i < kScanItems; ++i)
            if (base + i < n) {
                acc += in[base + i];
                mx = max(mx, in[base + i]);
            }
    }
    int total;
    block_exclusive_scan(acc, lds, &total);
    if (threadIdx.x == 0) sums[blockIdx.x] = total;
    if (max_out) {
        mx = wave_max(mx);
        // one address for the whole grid: skip atomics the maximum already covers
        if ((threadIdx.x & (kWave - 1)) == 0 && mx > *(volatile int32_t*)max_out) atomicMax(max_out, mx);
    }
}

__global__ __launch_bounds__(kScanThreads) void k_tile_scan(const int32_t* __restrict__ in,
                                                             int64_t n, const int32_t* __restrict__ base_of_tile,
                                                             int32_t* __restrict__ out, const int32_t* gate) {
    if (gated(gate)) return;
    __shared__ int lds[kScanThreads / kWave + 1];
    const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
    int v[kScanItems];
    const bool full = base + kScanItems <= n;
    if (full) {
        const int4* p = reinterpret_cast<const int4*>(in + base);
#pragma unroll
        for (int i = 0; i < kScanItems / 4; ++i) {
            int4 q = p[i];
            v[4 * i] = q.x; v[4 * i + 1] = q.y; v[4 * i + 2] = q.z; v[4 * i + 3] = q.w;
        }
    } else {
#pragma unroll
        for (int i = 0; i < kScanItems; ++i) v[i] = (base + i < n) ? in[base + i] : 0;
    }
    int acc = 0;
#pragma unroll
    for (int i = 0; i < kScanItems; ++i) acc += v[i];
    int total;
    int run = block_exclusive_scan(acc, lds, &total) + base_of_tile[blockIdx.x];
    if (full) {
        int4* o = reinterpret_cast<int4*>(out + base);
#pragma unroll
        for (int i = 0; i < kScanItems / 4; ++i) {
            int4 q;
            q.x = run; run += v[4 * i];
            q.y = run; run += v[4 * i + 1];
            q.z = run; run += v[4 * i + 2];
            q.w = run; run += v[4 * i + 3];
            o[i] = q;
        }
    } else {
        for (int i = 0; i < kScanItems; ++i) {
            if (base + i < n) out[base + i] = run;
            run += v[i];
        }
    }
    if (blockIdx.x == gridDim.x - 1 && threadIdx.x == 0)
        out[n] = base_of_tile[blockIdx.x] + total;
}

// Single-block scan for short inputs (n <= kScanTile): out[0..n].
__global__ __launch_bounds__(kScanThreads) void k_small_scan(const int32_t* __restrict__ in, int64_t n,
                                                              int32_t* __restrict__ out, int32_t* __restrict__ max_out,
                                                              const int32_t* gate) {
    if (gated(gate)) return;
    __shared__ int lds[kScanThreads / kWave + 1];
    const int64_t base = (int64_t)threadIdx.x * kScanItems;
    int v[kScanItems];
    int acc = 0, mx = 0;
#pragma unroll
    for (int i = 0; i < kScanItems; ++i) {
        v[i] = (base + i < n) ? in[base + i] : 0;
        acc += v[i];
        mx = max(mx, v[i]);
    }
    int total;
    int run = block_exclusive_scan(acc, lds, &total);
    for (int i = 0; i < kScanItems; ++i) {
        if (base + i < n) out[base + i] = run;
        run += v[i];
    }
    if (threadIdx.x == 0) out[n] = total;
    if (max_out) {
        mx = wave_max(mx);
        // one address for the whole grid: skip atomics the maximum already covers
        if ((threadIdx.x & (kWave - 1)) == 0 && mx > *(volatile int32_t*)max_out) atomicMax(max_out, mx);
    }
}

inline int64_t round16(int64_t x) { return (x + 15) / 16 * 16; }

// out[0] += sum of in (64-bit), out[1] = min(out[1], smallest value)
__global__ __launch_bounds__(kScanThreads) void k_count_check(const int32_t* __restrict__ in, int64_t n,
                                                               long long* __restrict__ out) {
    long long sum = 0;
    int mn = 0x7fffffff;
    for (int64_t i = (int64_t)blockIdx.x * kScanThreads + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * kScanThreads) {
        const int v = in[i];
        sum += v;
        mn = min(mn, v);
    }
#pragma unroll
    for (int d = kWave / 2; d > 0; d >>= 1) {
        sum += __shfl_xor(sum, d, kWave);
        mn = min(mn, __shfl_xor(mn, d, kWave));
    }
    if ((threadIdx.x & (kWave - 1)) == 0) {
        atomicAdd(reinterpret_cast<unsigned long long*>(&out[0]), (unsigned long long)sum);
        atomicMin(&out[1], (long long)mn);
    }
}

}  // namespace

void launch_count_check(const int32_t* counts, int64_t n, long long* out, hipStream_t s) {
    const unsigned blocks = (unsigned)std::min<int64_t>(1024, std::max<int64_t>(1, (n + kScanThreads - 1) / kScanThreads));
    hipLaunchKernelGGL(k_count_check, dim3(blocks), dim3(kScanThreads), 0, s, counts, n, out);
}

size_t scan_workspace_bytes(int64_t n) {
    size_t bytes = 0;
    int64_t m = n;
    while (m > kScanTile) {
        int64_t nb = (m + kScanTile - 1) / kScanTile;
        bytes += (size_t)(round16(nb) + round16(nb + 1)) * sizeof(int32_t);
        m = nb;
    }
    return bytes + 256;
}

void exclusive_scan_i32(const int32_t* in, int32_t* out, int64_t n, void* ws, hipStream_t s, int32_t* max_out,
                        const int32_t* gate) {
    if (n <= kScanTile) {
        hipLaunchKernelGGL(k_small_scan, dim3(1), dim3(kScanThreads), 0, s, in, n, out, max_out, gate);
        return;
    }
    const int64_t nb = (n + kScanTile - 1) / kScanTile;
    // keep every array 64-byte aligned: the tile kernels use 16-byte vectors
    int32_t* sums = static_cast<int32_t*>(ws);
    int32_t* sums_scan = sums + round16(nb);
    void* rest = sums_scan + round16(nb + 1);
    hipLaunchKernelGGL(k_tile_sums, dim3((unsigned)nb), dim3(kScanThreads), 0, s, in, n, sums, max_out, gate);
    exclusive_scan_i32(sums, sums_scan, nb, rest, s, nullptr, gate);
    hipLaunchKernelGGL(k_tile_scan, dim3((unsigned)nb), dim3(kScanThreads), 0, s, in, n, sums_scan, out, gate);
}

}  // namespace cube
