// Stable recompaction by cell (Sec. III-A: particles must stay cell-ordered
// for the position codec to locate their cell).  The new order is the stable
// counting sort of the old order by new canonical cell.
//
// Fast path (every particle moved at most one coarse cell per axis): the
// brick compaction below, from the records of the particles that changed
// cell, which the gather writes grouped by destination brick.
//
// General path: the new keys are sorted stably with the LSD radix sort and the
// planes are permuted.
#include <algorithm>

#include "common.h"

namespace cube {

namespace {

// Brick compaction from the gather's mover records.  One wave per gather
// brick D (tile-major numbering, XCD-aware).  The old storage order is the
// canonical cell order, so for a destination cell c the stable counting sort
// puts, in order of old index p: the particles arriving from cells stored
// before c, then c's own stayers, then the arrivals from cells stored after
// c.  Hence, with every arrival's old index p known,
//   stayer of c, k-th among them:  new_offset[c] + #(arrivals with p < off_old[c]) + k
//   arrival into c:                new_offset[c] + #(arrivals into c with smaller p)
//                                  + (p >= off_old[c] ? stayers of c : 0)
// with no distinction between tile faces, periodic wraps and interior cells.
// The arrivals are the records of class "towards D" of D and its 26
// neighbours (the gather groups each brick's records by class); stayers are
// D's own particles with move code 13, ranked by a wave scan per 64.
// The work per brick is a handful of short dependent phases, so every load
// of a phase is issued before the first is used, and a small LDS footprint
// keeps many bricks in flight per CU.  Bricks with more arrivals than the
// LDS list holds rank them from the records in memory (slower, same result).
constexpr int kKThreads = kWave;
constexpr int kInCap = 192;

template <int R>
__global__ __launch_bounds__(kKThreads) void k_compact_brick(Geom g, const int32_t* __restrict__ off_old,
                                                             const int32_t* __restrict__ off_new,
                                                             const uint8_t* __restrict__ dir,
                                                             const uint4* __restrict__ ment,
                                                             const int32_t* __restrict__ mhdr, Planes src,
                                                             Planes dst, const StepScalars* sc) {
    if (*(volatile const int32_t*)&sc->halt) return;
    constexpr int BXc = kGBX / R, BYc = kGBY / R, BZc = kGBZ / R;
    constexpr int NROW = BYc * BZc, NCELL = BXc * NROW;
    static_assert(NCELL <= kWave && NROW <= 8 && BXc <= 8, "brick shape");
    __shared__ int s_oo[NROW][BXc + 1], s_on[NROW][BXc + 1];
    __shared__ int s_rowpref[NROW + 1];
    __shared__ int s_abefore[NCELL], s_stay[NCELL];
    __shared__ int s_lbase[27], s_lpref[28];
    __shared__ uint4 s_in[kInCap];

    const int lane = (int)threadIdx.x;
    const int64_t lin = xcd_logical_block();
    const int nbx = g.T / kGBX, nby = g.T / kGBY, nbz = g.T / kGBZ, bpt = nbx * nby * nbz;
    const int tile = (int)(lin / bpt), b = (int)(lin - (int64_t)tile * bpt);
    const int tx = tile % g.nt, ty = (tile / g.nt) % g.nt, tz = tile / (g.nt * g.nt);
    // global brick coordinates and the brick's first coarse cell
    const int gb[3] = {tx * nbx + b % nbx, ty * nby + (b / nbx) % nby, tz * nbz + b / (nbx * nby)};
    const int c0[3] = {gb[0] * BXc, gb[1] * BYc, gb[2] * BZc};
    const int NB[3] = {g.nt * nbx, g.nt * nby, g.nt * nbz};

    for (int t = lane; t < NROW * (BXc + 1); t += kKThreads) {
        const int r = t / (BXc + 1), j = t - r * (BXc + 1);
        const int64_t c = canon(g, c0[0], c0[1] + r % BYc, c0[2] + r / BYc) + j;
        s_oo[r][j] = off_old[c];
        s_on[r][j] = off_new[c];
    }
    // the brick at offset o sends the records of class 26 - o here
    int cnt = 0;
    if (lane < 27) {
        const int o = lane;
        int sb[3] = {gb[0] + o % 3 - 1, gb[1] + (o / 3) % 3 - 1, gb[2] + o / 9 - 1};
#pragma unroll
        for (int k = 0; k < 3; ++k) sb[k] = sb[k] < 0 ? sb[k] + NB[k] : (sb[k] >= NB[k] ? sb[k] - NB[k] : sb[k]);
        const int stile = sb[0] / nbx + g.nt * (sb[1] / nby + g.nt * (sb[2] / nbz));
        const int sbl = sb[0] % nbx + nbx * (sb[1] % nby + nby * (sb[2] % nbz));
        const int32_t* h = mhdr + ((int64_t)stile * bpt + sbl) * kHdrInts;
        const int c = 26 - o;
        const int lo = h[1 + c], hi = h[2 + c];
        s_lbase[o] = h[0] + lo;
        cnt = hi - lo;
    }
    {
        const int incl = wave_inclusive_scan(cnt);
        if (lane < 27) s_lpref[lane] = incl - cnt;
        if (lane == 26) s_lpref[27] = incl;
    }
    if (lane < NCELL) {
        s_abefore[lane] = 0;
        s_stay[lane] = 0;
    }
    __syncthreads();
    if (lane == 0) {
        s_rowpref[0] = 0;
        for (int r = 0; r < NROW; ++r) s_rowpref[r + 1] = s_rowpref[r] + (s_oo[r][BXc] - s_oo[r][0]);
    }
    const int nin = s_lpref[27];
    const bool listed = nin <= kInCap;
    auto arrival = [&](int i) -> uint4 {
        const int l = find_cell_fixed<5>(s_lpref, 27, i);
        return ment[s_lbase[l] + (i - s_lpref[l])];
    };
    if (listed) {
        constexpr int UC = 3;                      // record loads in flight per lane
        for (int i0 = 0; i0 < nin; i0 += UC * kKThreads) {
            uint4 rec[UC];
#pragma unroll
            for (int u = 0; u < UC; ++u) {
                const int i = i0 + u * kKThreads + lane;
                if (i < nin) rec[u] = arrival(i);
            }
#pragma unroll
            for (int u = 0; u < UC; ++u) {
                const int i = i0 + u * kKThreads + lane;
                if (i < nin) s_in[i] = rec[u];
            }
        }
    }
    __syncthreads();
    auto oo_of = [&](int d) { return s_oo[d / BXc][d % BXc]; };
    // arrivals from cells stored before each destination cell
    for (int i = lane; i < nin; i += kKThreads) {
        const uint4 rec = listed ? s_in[i] : arrival(i);
        const int d = (int)(rec.y & 255);
        if ((int)rec.x < oo_of(d)) atomicAdd(&s_abefore[d], 1);
    }
    __syncthreads();

    // own particles in storage order, U chunks of 64 per round with every
    // load of the round in flight before the first is used: stayers keep
    // their order within their cell and are written straight to their slot
    const int nown = s_rowpref[NROW];
    const bool cp_u = src.u[0] != nullptr, cp_v = src.v[0] != nullptr, cp_id = dst.ids != nullptr;
    constexpr int U = 4;
    for (int base0 = 0; base0 < nown; base0 += U * kKThreads) {
        int pv[U], rowv[U], xv[U], code[U];
        uint32_t mb[U], ub[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int e = base0 + u * kKThreads + lane;
            pv[u] = -1;
            rowv[u] = 0;
            xv[u] = 0;
            code[u] = 0;
            mb[u] = 0;
            ub[u] = 0;
            if (e < nown) {
                const int row = find_cell_fixed<3>(s_rowpref, NROW, e);
                const int p = s_oo[row][0] + (e - s_rowpref[row]);
                pv[u] = p;
                rowv[u] = row;
                xv[u] = find_cell_fixed<3>(s_oo[row], BXc, p);
                code[u] = dir[p];
                // the planes are read for every particle: waiting for the code
                // first would cost a round trip, and movers are few
                mb[u] = (uint32_t)src.m[0][p] | ((uint32_t)src.m[1][p] << 8) | ((uint32_t)src.m[2][p] << 16);
                if (cp_u)
                    ub[u] = (uint32_t)(uint8_t)src.u[0][p] | ((uint32_t)(uint8_t)src.u[1][p] << 8) |
                            ((uint32_t)(uint8_t)src.u[2][p] << 16);
            }
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int base = base0 + u * kKThreads;
            if (base >= nown) break;
            const int e = base + lane;
            const int row = rowv[u], x = xv[u], p = pv[u];
            const int cl = x + BXc * row;
            int stay = 0, first = 0, cell_end = 0;
            if (e < nown) {
                stay = code[u] == 13 ? 1 : 0;
                // chunk positions of this particle's cell
                const int cell_e = s_rowpref[row] + (s_oo[row][x] - s_oo[row][0]);
                cell_end = s_rowpref[row] + (s_oo[row][x + 1] - s_oo[row][0]);
                first = max(cell_e, base) - base;
            }
            const int incl = wave_inclusive_scan(stay);
            const int before_first = __shfl(incl, max(first - 1, 0), kWave);
            const int before = first > 0 ? before_first : 0;
            const int k = s_stay[cl] + (incl - stay - before);
            if (e < nown && stay) {
                const int o = s_on[row][x] + s_abefore[cl] + k;
                if (o >= 0 && o < g.n) {
#pragma unroll
                    for (int a = 0; a < 3; ++a) {
                        dst.m[a][o] = (uint8_t)(mb[u] >> (8 * a));
                        if (cp_u) dst.u[a][o] = (int8_t)(ub[u] >> (8 * a));
                        if (cp_v) dst.v[a][o] = src.v[a][p];
                    }
                    if (cp_id) dst.ids[o] = src.ids[p];
                }
            }
            __syncthreads();
            // the last particle of each cell's run in this chunk carries the count on
            if (e < nown && (e == nown - 1 || lane == kKThreads - 1 || e + 1 == cell_end))
                s_stay[cl] += incl - before;
            __syncthreads();
        }
    }

    // arrivals: rank among the arrivals into the same cell by old index
    for (int i = lane; i < nin; i += kKThreads) {
        const uint4 rec = listed ? s_in[i] : arrival(i);
        const int d = (int)(rec.y & 255), p = (int)rec.x;
        int rank = 0;
        for (int j = 0; j < nin; ++j) {
            const uint4 q = listed ? s_in[j] : arrival(j);
            rank += ((int)(q.y & 255) == d && q.x < rec.x) ? 1 : 0;
        }
        const int row = d / BXc, x = d - row * BXc;
        const int o = s_on[row][x] + rank + (p >= s_oo[row][x] ? s_stay[d] : 0);
        if (o < 0 || o >= g.n || p < 0 || p >= g.n) continue;
        dst.m[0][o] = (uint8_t)(rec.z & 255);
        dst.m[1][o] = (uint8_t)((rec.z >> 8) & 255);
        dst.m[2][o] = (uint8_t)((rec.z >> 16) & 255);
        if (cp_u) {
            dst.u[0][o] = (int8_t)(rec.w & 255);
            dst.u[1][o] = (int8_t)((rec.w >> 8) & 255);
            dst.u[2][o] = (int8_t)((rec.w >> 16) & 255);
        }
        if (cp_v)
#pragma unroll
            for (int a = 0; a < 3; ++a) dst.v[a][o] = src.v[a][p];
        if (cp_id) dst.ids[o] = src.ids[p];
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
        if (src.u[0]) dst.u[a][j] = src.u[a][p];
        if (src.v[0]) dst.v[a][j] = src.v[a][p];
    }
    if (dst.ids) dst.ids[j] = src.ids[p];
}

}  // namespace

int64_t compact_bricks(const Geom& g) {
    return (int64_t)g.ntiles * (g.T / kGBX) * (g.T / kGBY) * (g.T / kGBZ);
}

void launch_compact_bricks(const Geom& g, const int32_t* offsets_old, const int32_t* offsets_new,
                           const uint8_t* dir, const uint4* ment, const int32_t* mhdr, Planes src, Planes dst,
                           const StepScalars* sc, hipStream_t s) {
    const dim3 grid((unsigned)compact_bricks(g));
    if (g.r == 4)
        hipLaunchKernelGGL(k_compact_brick<4>, grid, dim3(kKThreads), 0, s, g, offsets_old, offsets_new, dir, ment,
                           mhdr, src, dst, sc);
    else
        hipLaunchKernelGGL(k_compact_brick<8>, grid, dim3(kKThreads), 0, s, g, offsets_old, offsets_new, dir, ment,
                           mhdr, src, dst, sc);
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
