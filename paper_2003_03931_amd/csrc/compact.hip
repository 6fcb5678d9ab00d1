// Stable recompaction by cell (Sec. III-A: particles must stay cell-ordered
// for the position codec to locate their cell).  The new order is the stable
// counting sort of the old order by new canonical cell.
//
// Fast path (every particle moved at most one coarse cell per axis): one
// workgroup owns a 4^3 block of destination cells.  Its particles can only
// come from the 6^3 halo of source cells around it, so it histograms the move
// codes of those sources (27 directions), orders each destination's 27 source
// cells by canonical index, and places every incoming particle at
//   new_offset[dest] + (particles from earlier sources) + (rank among the
//   earlier same-direction particles of its own source cell).
// Deterministic, no global atomics.  Needs N_c to be a multiple of 4 and >= 6.
//
// General path: the new keys are sorted stably with the LSD radix sort and the
// planes are permuted.
#include "common.h"

namespace cube {

namespace {

constexpr int kCB = 4;                         // destination block side
constexpr int kHalo = kCB + 2;                 // source window side
constexpr int kNH = kHalo * kHalo * kHalo;     // 216 source cells
constexpr int kND = kCB * kCB * kCB;           // 64 destination cells

__global__ __launch_bounds__(256) void k_compact_fast(Geom g, const int32_t* __restrict__ off_old,
                                                       const int32_t* __restrict__ off_new,
                                                       const uint8_t* __restrict__ dir, Planes src, Planes dst) {
    __shared__ int h_canon[kNH], h_start[kNH], h_pref[kNH + 1];
    __shared__ int hist[kNH][27];
    __shared__ int pre[kND][27];
    __shared__ int d_off[kND];
    __shared__ int s_scan[256 / kWave + 1];

    const int nb = g.Nc / kCB;
    const int b = blockIdx.x;
    const int B0[3] = {(b % nb) * kCB, ((b / nb) % nb) * kCB, (b / (nb * nb)) * kCB};

    int cnt = 0;
    if (threadIdx.x < kNH) {
        const int h = threadIdx.x;
        const int hx = h % kHalo, hy = (h / kHalo) % kHalo, hz = h / (kHalo * kHalo);
        const int64_t c = canon(g, wrapi(B0[0] + hx - 1, g.Nc), wrapi(B0[1] + hy - 1, g.Nc),
                                wrapi(B0[2] + hz - 1, g.Nc));
        h_canon[h] = (int)c;
        const int st = off_old[c];
        cnt = off_old[c + 1] - st;
        h_start[h] = st;
#pragma unroll
        for (int d = 0; d < 27; ++d) hist[h][d] = 0;
    }
    if (threadIdx.x < kND) {
        const int e = threadIdx.x;
        const int ex = e % kCB, ey = (e / kCB) % kCB, ez = e / (kCB * kCB);
        d_off[e] = off_new[canon(g, B0[0] + ex, B0[1] + ey, B0[2] + ez)];
    }
    int total;
    const int pref = block_exclusive_scan(cnt, s_scan, &total);
    if (threadIdx.x < kNH) h_pref[threadIdx.x] = pref;
    if (threadIdx.x == 0) h_pref[kNH] = total;
    __syncthreads();

    // 27-direction histogram of every source cell
    for (int e = threadIdx.x; e < total; e += blockDim.x) {
        const int s = find_cell(h_pref, kNH, e);
        const int p = h_start[s] + (e - h_pref[s]);
        const int d = dir[p];
        if (d < 27) atomicAdd(&hist[s][d], 1);
    }
    __syncthreads();

    // pre[dest][d]: particles arriving from sources that precede source(dest, d)
    for (int e = threadIdx.x; e < kND * 27; e += blockDim.x) {
        const int dest = e / 27, d = e % 27;
        const int ex = dest % kCB + 1, ey = (dest / kCB) % kCB + 1, ez = dest / (kCB * kCB) + 1;
        const int hs = (ex - (d % 3 - 1)) + kHalo * ((ey - ((d / 3) % 3 - 1)) + kHalo * (ez - (d / 9 - 1)));
        const int my = h_canon[hs];
        int acc = 0;
        for (int d2 = 0; d2 < 27; ++d2) {
            const int hs2 =
                (ex - (d2 % 3 - 1)) + kHalo * ((ey - ((d2 / 3) % 3 - 1)) + kHalo * (ez - (d2 / 9 - 1)));
            if (h_canon[hs2] < my) acc += hist[hs2][d2];
        }
        pre[dest][d] = acc;
    }
    __syncthreads();

    // place every particle whose destination lies in this block
    for (int e = threadIdx.x; e < total; e += blockDim.x) {
        const int s = find_cell(h_pref, kNH, e);
        const int p = h_start[s] + (e - h_pref[s]);
        const int d = dir[p];
        if (d >= 27) continue;
        const int sx = s % kHalo, sy = (s / kHalo) % kHalo, sz = s / (kHalo * kHalo);
        const int ex = sx + (d % 3 - 1) - 1, ey = sy + ((d / 3) % 3 - 1) - 1, ez = sz + (d / 9 - 1) - 1;
        if (ex < 0 || ex >= kCB || ey < 0 || ey >= kCB || ez < 0 || ez >= kCB) continue;
        const int dest = ex + kCB * (ey + kCB * ez);
        int rank = 0;
        for (int q = h_start[s]; q < p; ++q) rank += (dir[q] == d);
        const int64_t o = (int64_t)d_off[dest] + pre[dest][d] + rank;
        if (o < 0 || o >= g.n) continue;          // inconsistent counts: never write out of range
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            dst.m[a][o] = src.m[a][p];
            dst.u[a][o] = src.u[a][p];
        }
        if (dst.ids) dst.ids[o] = src.ids[p];
    }
}

// keys of the general path: new canonical cell of every particle, old order
__global__ __launch_bounds__(256) void k_general_keys(Geom g, const int32_t* __restrict__ offsets,
                                                       const uint8_t* __restrict__ dir,
                                                       const uint32_t* __restrict__ far_key, uint32_t* __restrict__ key,
                                                       uint32_t* __restrict__ idx) {
    extern __shared__ int offs[];
    const Chunk ch = chunk_of(g, blockIdx.x);
    for (int j = threadIdx.x; j <= g.Tc; j += blockDim.x) offs[j] = offsets[ch.c0 + j];
    __syncthreads();
    for (int p = offs[0] + threadIdx.x; p < offs[g.Tc]; p += blockDim.x) {
        const int d = dir[p];
        uint32_t k;
        if (d < 27) {
            const int j = find_cell(offs, g.Tc, p);
            k = (uint32_t)canon(g, wrapi(ch.cx0 + j + d % 3 - 1, g.Nc), wrapi(ch.cy + (d / 3) % 3 - 1, g.Nc),
                                wrapi(ch.cz + d / 9 - 1, g.Nc));
        } else {
            k = far_key[p];
        }
        key[p] = k;
        idx[p] = (uint32_t)p;
    }
}

__global__ void k_permute(const uint32_t* __restrict__ perm, Planes src, Planes dst, int64_t n) {
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n) return;
    const uint32_t p = perm[j];
    if (p >= n) return;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        dst.m[a][j] = src.m[a][p];
        dst.u[a][j] = src.u[a][p];
    }
    if (dst.ids) dst.ids[j] = src.ids[p];
}

}  // namespace

void launch_compact_fast(const Geom& g, const int32_t* offsets_old, const int32_t* offsets_new, const uint8_t* dir,
                         Planes src, Planes dst, hipStream_t s) {
    const int nb = g.Nc / kCB;
    hipLaunchKernelGGL(k_compact_fast, dim3(nb * nb * nb), dim3(256), 0, s, g, offsets_old, offsets_new, dir, src,
                       dst);
}

void launch_general_keys(const Geom& g, const int32_t* offsets_old, const uint8_t* dir, const uint32_t* far_key,
                         uint32_t* key, uint32_t* idx, hipStream_t s) {
    const int64_t chunks = g.ncells / g.Tc;
    hipLaunchKernelGGL(k_general_keys, dim3((unsigned)chunks), dim3(256), (g.Tc + 1) * sizeof(int), s, g,
                       offsets_old, dir, far_key, key, idx);
}

void launch_permute_planes(const uint32_t* perm, Planes src, Planes dst, int64_t n, hipStream_t s) {
    hipLaunchKernelGGL(k_permute, dim3(grid1d(n, 256)), dim3(256), 0, s, perm, src, dst, n);
}

}  // namespace cube
