// Device helpers shared by the kernels of libcube.so (wavefront-64 scans and
// reductions, checked HIP launches).
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

#include "internal.h"

namespace cube {

constexpr int kWave = 64;

// Inclusive scan inside one 64-lane wavefront.
__device__ inline int wave_inclusive_scan(int v) {
    const int lane = threadIdx.x & (kWave - 1);
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
        int t = __shfl_up(v, d, kWave);
        if (lane >= d) v += t;
    }
    return v;
}

// Exclusive scan over the whole block (blockDim.x a multiple of 64, <= 1024).
// lds needs blockDim.x / 64 + 1 ints.  Returns the exclusive prefix of v and
// writes the block total to *total.
__device__ inline int block_exclusive_scan(int v, int* lds, int* total) {
    const int lane = threadIdx.x & (kWave - 1);
    const int wid = threadIdx.x / kWave;
    const int nw = blockDim.x / kWave;
    int inc = wave_inclusive_scan(v);
    if (lane == kWave - 1) lds[wid] = inc;
    __syncthreads();
    if (threadIdx.x == 0) {
        int acc = 0;
        for (int w = 0; w < nw; ++w) {
            int t = lds[w];
            lds[w] = acc;
            acc += t;
        }
        lds[nw] = acc;
    }
    __syncthreads();
    int res = inc - v + lds[wid];
    *total = lds[nw];
    __syncthreads();
    return res;
}

// The same scan with barriers that order LDS alone, for callers whose global
// stores still in flight need not complete first.  Defined after lds_barrier.
__device__ inline int block_exclusive_scan_lds(int v, int* lds, int* total);

__device__ inline int wave_max(int v) {
#pragma unroll
    for (int d = kWave / 2; d > 0; d >>= 1) v = max(v, __shfl_xor(v, d, kWave));
    return v;
}

__device__ inline int wave_sum(int v) {
#pragma unroll
    for (int d = kWave / 2; d > 0; d >>= 1) v += __shfl_xor(v, d, kWave);
    return v;
}

__device__ inline double wave_sum_d(double v) {
#pragma unroll
    for (int d = kWave / 2; d > 0; d >>= 1) v += __shfl_xor(v, d, kWave);
    return v;
}

inline unsigned grid1d(int64_t work, int per_block) {
    int64_t b = (work + per_block - 1) / per_block;
    return (unsigned)(b < 1 ? 1 : b);
}

}  // namespace cube

namespace cube {

// A chunk is one x-row of coarse cells inside one tile: Tc consecutive cells
// in canonical order, hence one contiguous particle range.
struct Chunk {
    int cx0, cy, cz;   // global coarse coords of the chunk's first cell
    int64_t c0;        // canonical index of that cell
    int tile;          // tile index
    int ly, lz;        // tile-local row coordinates
};

__device__ inline Chunk chunk_of(const Geom& g, int64_t q) {
    const int Tc = g.Tc;
    const int64_t per_tile = (int64_t)Tc * Tc;
    Chunk c;
    c.tile = (int)(q / per_tile);
    const int rem = (int)(q - (int64_t)c.tile * per_tile);
    c.ly = rem % Tc;
    c.lz = rem / Tc;
    const int tx = c.tile % g.nt, ty = (c.tile / g.nt) % g.nt, tz = c.tile / (g.nt * g.nt);
    c.cx0 = tx * Tc;
    c.cy = ty * Tc + c.ly;
    c.cz = tz * Tc + c.lz;
    c.c0 = q * Tc;
    return c;
}

// Index j with offs[j] <= p < offs[j+1] among offs[0..len] (offs[0] <= p < offs[len]).
__device__ inline int find_cell(const int* offs, int len, int p) {
    int lo = 0, hi = len;   // invariant offs[lo] <= p < offs[hi]
    while (hi - lo > 1) {
        int mid = (lo + hi) >> 1;
        if (offs[mid] <= p) lo = mid; else hi = mid;
    }
    return lo;
}

// The same search with a fixed number of steps (len <= 2^LOG2): the largest
// index i < len with offs[i] <= p.  With no data-dependent trip count, the
// searches of several unrolled elements overlap their LDS latencies.
template <int LOG2>
__device__ __forceinline__ int find_cell_fixed(const int* offs, int len, int p) {
    int lo = 0;
#pragma unroll
    for (int step = 1 << (LOG2 - 1); step > 0; step >>= 1) {
        const int mid = lo + step;
        if (mid < len && offs[mid] <= p) lo = mid;
    }
    return lo;
}

}  // namespace cube

namespace cube {

// Copy `total` elements from global to LDS with U independent loads in flight
// per thread: lds[lidx(e)] = glob[gidx(e)] for e in [0, total).  Issuing the
// loads of a batch before any LDS store keeps the memory pipe full instead of
// paying one full latency per element.
template <int NT, int U, class T, class FG, class FL>
__device__ __forceinline__ void stage_to_lds(int total, const T* __restrict__ glob, T* lds, FG gidx, FL lidx) {
    for (int base = 0; base < total; base += NT * U) {
        T tmp[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int e = base + u * NT + (int)threadIdx.x;
            if (e < total) tmp[u] = glob[gidx(e)];
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int e = base + u * NT + (int)threadIdx.x;
            if (e < total) lds[lidx(e)] = tmp[u];
        }
    }
}

}  // namespace cube

namespace cube {

constexpr int kXcds = 8;

// Workgroups are handed to the 8 XCDs round-robin (linear id mod 8).  This
// maps the linear id to a logical block so that each XCD receives one
// contiguous range of logical blocks: neighbouring blocks, which share
// particle ranges, offsets and halos, then share one L2.
__device__ __forceinline__ int64_t xcd_logical_block() {
    const int64_t nb = (int64_t)gridDim.x * gridDim.y;
    const int64_t bid = blockIdx.x + (int64_t)gridDim.x * blockIdx.y;
    const int64_t per = nb / kXcds, rem = nb % kXcds;
    const int64_t x = bid % kXcds, k = bid / kXcds;
    return x * per + (x < rem ? x : rem) + k;
}

// Workgroup barrier that orders LDS only.  __syncthreads() also releases
// global memory, which makes every wave wait for its own outstanding global
// stores at the barrier; a persistent loop that stores one item's results
// and meets at the top of the next item would expose the store latency on
// every item.  Use this where the barrier protects LDS alone.
__device__ __forceinline__ void lds_barrier() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

__device__ inline int block_exclusive_scan_lds(int v, int* lds, int* total) {
    const int lane = threadIdx.x & (kWave - 1);
    const int wid = threadIdx.x / kWave;
    const int nw = blockDim.x / kWave;
    int inc = wave_inclusive_scan(v);
    if (lane == kWave - 1) lds[wid] = inc;
    lds_barrier();
    if (threadIdx.x == 0) {
        int acc = 0;
        for (int w = 0; w < nw; ++w) {
            int t = lds[w];
            lds[w] = acc;
            acc += t;
        }
        lds[nw] = acc;
    }
    lds_barrier();
    int res = inc - v + lds[wid];
    *total = lds[nw];
    lds_barrier();
    return res;
}

}  // namespace cube

namespace cube {

// Eq. (3) decode of the cell-mean velocity codec: v_c + sigma tan(u pi / 255)
// (table entry u + 127), in FP64 and in that order.  The byte -128, which no
// encoder writes, reads as -127.
__device__ __forceinline__ double vc_decode(float vc, double sigma, const double* tab, int u) {
    return (double)vc + sigma * tab[max(u, -127) + 127];
}

}  // namespace cube
