// Cloud-in-cell mass assignment (Sec. II: density by interpolating particles
// onto a mesh; the tile's fine mesh is the tile plus its buffer) on the
// fixed-point positions of Eq. (2).
//
// Owner-computes: every workgroup owns a cube of target cells, pulls the
// particles of the coarse cells that can reach it (its own plus one coarse
// cell on each face) straight from the cell-ordered arrays, accumulates the
// exact CIC weights in LDS as 64-bit integers and writes each target cell
// once -- no global atomics, bit-reproducible.
//
// Exactness: a coordinate in target-cell units is P / D with P = 2(c 256 + m)+1
// and D = 512 / (target cells per coarse cell), so every CIC weight is an
// integer multiple of 1/D per axis and of 1/D^3 in 3-D.  The FP32 output is
// round(acc / D^3 / cell_volume - 1), the single rounding of the exact value.
// A target cell gathers particles of at most one 2 x 2 x 2 block of coarse
// cells, each weight at most D^3, so 32-bit accumulators are exact whenever
// D^3 times the largest such block count is below 2^32 (the caller checks the
// state's block counts); otherwise 64-bit.
//
// The brick kernel serves the periodic single-tile mesh and the diagnostic
// mesh; tile meshes of a tiled box use the z-marching form further down.
#include "common.h"

namespace cube {

namespace {

enum DepositMode { DEP_COARSE = 0, DEP_FINE_TILED = 1, DEP_FINE_PERIODIC = 2, DEP_DIAG = 3 };

constexpr int kDepThreads = 256;

// MAXSRC bounds the source window, (BW / cpc + 2)^3 coarse cells; MAPCAP is
// the number of window particles whose source cell is looked up from a
// per-particle map (larger windows fall back to a binary search).
template <int BW, int MODE, class ACC, int MAXSRC, int MAPCAP>
__global__ __launch_bounds__(kDepThreads) void k_deposit(Geom g, const int32_t* __restrict__ offsets, Planes p,
                                                          float* __restrict__ out, int M, int cpc, int log2D,
                                                          double scale, int tile0) {
    static_assert(MAXSRC <= 1024, "fixed-step search over the source window");
    __shared__ __align__(16) ACC acc[BW * BW * BW];
    __shared__ int s_start[MAXSRC];
    __shared__ int s_pref[MAXSRC + 1];
    __shared__ int s_rel[MAXSRC];                // window coordinates + 1, 8 bits each
    __shared__ uint16_t s_map[MAPCAP];
    __shared__ int s_scan[kDepThreads / kWave + 1];

    const int nbx = (M + BW - 1) / BW;
    const int64_t lb = xcd_logical_block();
    const int b = (int)(lb % gridDim.x);        // block within the mesh
    const int ky = (int)(lb / gridDim.x);       // tile within the batch
    const int T0[3] = {(b % nbx) * BW, ((b / nbx) % nbx) * BW, (b / (nbx * nbx)) * BW};
    const int bw[3] = {min(BW, M - T0[0]), min(BW, M - T0[1]), min(BW, M - T0[2])};
    int nsa[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) nsa[k] = (bw[k] + cpc - 1) / cpc + 2;
    const int nsrc = nsa[0] * nsa[1] * nsa[2];
    // source frame origin (coarse cells): one cell before the block
    const int S0[3] = {T0[0] / cpc - 1, T0[1] / cpc - 1, T0[2] / cpc - 1};

    int tile = 0, box0[3] = {0, 0, 0};
    if (MODE == DEP_FINE_TILED) {
        tile = tile0 + ky;
        const int tx = tile % g.nt, ty = (tile / g.nt) % g.nt, tz = tile / (g.nt * g.nt);
        box0[0] = tx * g.Tc - g.hc;
        box0[1] = ty * g.Tc - g.hc;
        box0[2] = tz * g.Tc - g.hc;
    }

    static_assert(sizeof(acc) % sizeof(uint4) == 0, "accumulators are cleared 16 bytes at a time");
    for (int i = threadIdx.x; i < (int)(sizeof(acc) / sizeof(uint4)); i += kDepThreads)
        reinterpret_cast<uint4*>(acc)[i] = make_uint4(0u, 0u, 0u, 0u);

    // per-thread run of up to kPer source cells: counts, then a block scan
    constexpr int kPer = (MAXSRC + kDepThreads - 1) / kDepThreads;
    int my_cnt[kPer];
    int run = 0;
#pragma unroll
    for (int q = 0; q < kPer; ++q) {
        const int s = threadIdx.x * kPer + q;
        int cnt = 0;
        if (s < nsrc) {
            const int rx = s % nsa[0], ry = (s / nsa[0]) % nsa[1], rz = s / (nsa[0] * nsa[1]);
            s_rel[s] = rx | (ry << 8) | (rz << 16);
            int fc[3] = {S0[0] + rx, S0[1] + ry, S0[2] + rz};
            bool ok = true;
            if (MODE == DEP_FINE_TILED) {
#pragma unroll
                for (int k = 0; k < 3; ++k) {
                    ok = ok && fc[k] >= 0 && fc[k] < g.Fc;
                    fc[k] += box0[k];
                }
            }
            if (ok) {
                const int64_t c = canon(g, wrapi(fc[0], g.Nc), wrapi(fc[1], g.Nc), wrapi(fc[2], g.Nc));
                const int st = offsets[c];
                cnt = offsets[c + 1] - st;
                s_start[s] = st;
            } else {
                s_start[s] = 0;
            }
        }
        my_cnt[q] = cnt;
        run += cnt;
    }
    int total;
    int base = block_exclusive_scan(run, s_scan, &total);
    const bool mapped = total <= MAPCAP;
#pragma unroll
    for (int q = 0; q < kPer; ++q) {
        const int s = threadIdx.x * kPer + q;
        if (s < nsrc) {
            s_pref[s] = base;
            if (mapped)
                for (int j = 0; j < my_cnt[q]; ++j) s_map[base + j] = (uint16_t)s;
        }
        base += my_cnt[q];
    }
    if (threadIdx.x == 0) s_pref[nsrc] = total;
    __syncthreads();

    const int D = 1 << log2D;
    const int halfD = D >> 1;
    constexpr int U = 8;                       // particles per thread with loads in flight
    for (int base = 0; base < total; base += kDepThreads * U) {
        int mm[U][3], src_of[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int e = base + u * kDepThreads + threadIdx.x;
            src_of[u] = -1;
            if (e < total) {
                const int s = mapped ? (int)s_map[e] : find_cell_fixed<(MAXSRC <= 256 ? 8 : 10)>(s_pref, nsrc, e);
                const int pidx = s_start[s] + (e - s_pref[s]);
                src_of[u] = s;
#pragma unroll
                for (int k = 0; k < 3; ++k) mm[u][k] = p.m[k][pidx];
            }
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int s = src_of[u];
            if (s < 0) continue;
            const int rl = s_rel[s];
            const int rel[3] = {(rl & 255) - 1, ((rl >> 8) & 255) - 1, (rl >> 16) - 1};
            int i0[3];
            unsigned w1[3];
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                const int P = 2 * (rel[k] * 256 + mm[u][k]) + 1;   // units of 1/D target cells
                const int Pm = P - halfD;
                i0[k] = Pm >> log2D;                                // floor division
                w1[k] = (unsigned)(Pm & (D - 1));
            }
#pragma unroll
            for (int oz = 0; oz < 2; ++oz) {
                const int iz = i0[2] + oz;
                if (iz < 0 || iz >= bw[2]) continue;
                const unsigned wz = oz ? w1[2] : (unsigned)D - w1[2];
#pragma unroll
                for (int oy = 0; oy < 2; ++oy) {
                    const int iy = i0[1] + oy;
                    if (iy < 0 || iy >= bw[1]) continue;
                    // weights are at most D <= 512 per axis: 24-bit products
                    const unsigned wyz = (unsigned)__umul24(oy ? w1[1] : (unsigned)D - w1[1], wz);
#pragma unroll
                    for (int ox = 0; ox < 2; ++ox) {
                        const int ix = i0[0] + ox;
                        if (ix < 0 || ix >= bw[0]) continue;
                        const ACC w = (ACC)(unsigned)__umul24(ox ? w1[0] : (unsigned)D - w1[0], wyz);
                        if (w) atomicAdd(&acc[(iz * BW + iy) * BW + ix], w);
                    }
                }
            }
        }
    }
    __syncthreads();

    // exact value * scale - 1, rounded once to FP32
    if (MODE == DEP_FINE_TILED || MODE == DEP_FINE_PERIODIC) {
        // real mesh of tile ky: four x-consecutive cells per float4 store (the
        // block origin and the mesh side are multiples of 4, and so is bw[0])
        constexpr int Q = BW / 4;
        float* mesh = out + (int64_t)ky * M * M * M;
        for (int i4 = threadIdx.x; i4 < Q * BW * BW; i4 += kDepThreads) {
            const int ix = 4 * (i4 % Q), iy = (i4 / Q) % BW, iz = i4 / (Q * BW);
            if (ix >= bw[0] || iy >= bw[1] || iz >= bw[2]) continue;
            const ACC* a = &acc[(iz * BW + iy) * BW + ix];
            float4 v;
            v.x = (float)fma((double)a[0], scale, -1.0);
            v.y = (float)fma((double)a[1], scale, -1.0);
            v.z = (float)fma((double)a[2], scale, -1.0);
            v.w = (float)fma((double)a[3], scale, -1.0);
            const int64_t cell = (int64_t)(T0[0] + ix) + (int64_t)M * ((T0[1] + iy) + (int64_t)M * (T0[2] + iz));
            *reinterpret_cast<float4*>(mesh + cell) = v;
        }
        return;
    }
    for (int i = threadIdx.x; i < BW * BW * BW; i += kDepThreads) {
        const int ix = i % BW, iy = (i / BW) % BW, iz = i / (BW * BW);
        if (ix >= bw[0] || iy >= bw[1] || iz >= bw[2]) continue;
        const float v = (float)((double)acc[i] * scale - 1.0);
        const int64_t cell = (int64_t)(T0[0] + ix) + (int64_t)M * ((T0[1] + iy) + (int64_t)M * (T0[2] + iz));
        if (MODE == DEP_FINE_TILED || MODE == DEP_FINE_PERIODIC) {
            out[(int64_t)ky * M * M * M + cell] = v;     // real mesh of tile k
        } else {
            out[2 * cell] = v;
            out[2 * cell + 1] = 0.0f;
        }
    }
}

// The fine deposit of a batch of tile meshes, marching along z: a workgroup
// owns a BW x BW column of fine cells through the whole tile mesh and walks
// it in chunks of CZ fine planes (CZ / cpc coarse layers).  A chunk pulls the
// particles of its own coarse layers only (with one coarse cell on each side
// in x and y): its particles reach at most one plane below the chunk and one
// past it, so the accumulator holds CZ + 2 planes, and the two upper planes
// stay in LDS as the first two of the next chunk instead of being rebuilt
// from the layer above.  Per owned cell a chunk reads (BW / cpc + 2)^2 /
// (BW / cpc)^2 of the particles (1.56x for 32 x 32 columns at cpc = 4)
// against the brick's (BW / cpc + 2)^3 / (BW / cpc)^3 (3.4x for 16^3 bricks).
// The weights, the exactness and the single FP32 rounding are those of the
// brick kernel above.
template <int BW, int CZ, int NT, int U, class ACC, int MAXSRC, int MAPCAP>
__global__ __launch_bounds__(NT) void k_deposit_zm(Geom g, const int32_t* __restrict__ offsets, Planes p,
                                                    float* __restrict__ out, int cpc, int log2D, double scale,
                                                    int tile0) {
    static_assert(MAXSRC <= 1024, "fixed-step search over the source window");
    static_assert(BW % 4 == 0 && NT % kWave == 0, "float4 rows, whole waves");
    constexpr int NP = CZ + 2;                   // planes z0 - 1 .. z0 + CZ of chunk z0
    constexpr int PL = BW * BW;
    constexpr int kPer = (MAXSRC + NT - 1) / NT;
    __shared__ __align__(16) ACC acc[NP * PL];
    __shared__ int s_start[MAXSRC];
    __shared__ int s_pref[MAXSRC + 1];
    __shared__ int s_rel[MAXSRC];                // source cell: x, y from the column's ring, z in the chunk; 8 bits each
    __shared__ uint16_t s_map[MAPCAP];
    __shared__ int s_scan[NT / kWave + 1];

    const int M = g.F;
    const int nbx = (M + BW - 1) / BW;
    const int64_t lb = xcd_logical_block();
    const int b = (int)(lb % gridDim.x);        // column within the mesh
    const int ky = (int)(lb / gridDim.x);       // tile within the batch
    const int T0x = (b % nbx) * BW, T0y = (b / nbx) * BW;
    const int bwx = min(BW, M - T0x), bwy = min(BW, M - T0y);
    const int nsx = (bwx + cpc - 1) / cpc + 2, nsy = (bwy + cpc - 1) / cpc + 2;
    const int S0x = T0x / cpc - 1, S0y = T0y / cpc - 1;
    const int LC = CZ / cpc;                     // coarse layers per chunk
    const int nch = (g.Fc + LC - 1) / LC;
    const int tile = tile0 + ky;
    const int tx = tile % g.nt, ty = (tile / g.nt) % g.nt, tz = tile / (g.nt * g.nt);
    const int box0[3] = {tx * g.Tc - g.hc, ty * g.Tc - g.hc, tz * g.Tc - g.hc};
    float* mesh = out + (int64_t)ky * M * M * M;

    static_assert(sizeof(acc) % sizeof(uint4) == 0, "accumulators are cleared 16 bytes at a time");
    for (int i = threadIdx.x; i < (int)(sizeof(acc) / sizeof(uint4)); i += NT)
        reinterpret_cast<uint4*>(acc)[i] = make_uint4(0u, 0u, 0u, 0u);

    // particle ranges of chunk j's source cells, thread-owned runs of kPer
    int my_st[kPer], my_cnt[kPer];
    auto fetch = [&](int j) {
        const int c0 = j * LC, nsz = min(LC, g.Fc - c0);
        const int nsrc = nsx * nsy * nsz;
#pragma unroll
        for (int q = 0; q < kPer; ++q) {
            const int s = threadIdx.x * kPer + q;
            my_st[q] = 0;
            my_cnt[q] = 0;
            if (s < nsrc) {
                const int fx = S0x + s % nsx, fy = S0y + (s / nsx) % nsy, fz = c0 + s / (nsx * nsy);
                if (fx >= 0 && fx < g.Fc && fy >= 0 && fy < g.Fc) {
                    const int64_t c = canon(g, wrapi(fx + box0[0], g.Nc), wrapi(fy + box0[1], g.Nc),
                                            wrapi(fz + box0[2], g.Nc));
                    my_st[q] = offsets[c];
                    my_cnt[q] = offsets[c + 1] - my_st[q];
                }
            }
        }
    };
    fetch(0);

    const int D = 1 << log2D;
    const int halfD = D >> 1;
    const float scalef = (float)scale;           // a power of two
    constexpr int Q = BW / 4;
    for (int j = 0; j < nch; ++j) {
        const int nsrc = nsx * nsy * min(LC, g.Fc - j * LC);
        int run = 0;
#pragma unroll
        for (int q = 0; q < kPer; ++q) {
            const int s = threadIdx.x * kPer + q;
            if (s < nsrc) {
                s_rel[s] = (s % nsx) | (((s / nsx) % nsy) << 8) | ((s / (nsx * nsy)) << 16);
                s_start[s] = my_st[q];
            }
            run += my_cnt[q];
        }
        int total;
        int base = block_exclusive_scan_lds(run, s_scan, &total);
        const bool mapped = total <= MAPCAP;
#pragma unroll
        for (int q = 0; q < kPer; ++q) {
            const int s = threadIdx.x * kPer + q;
            if (s < nsrc) {
                s_pref[s] = base;
                if (mapped)
                    for (int e = 0; e < my_cnt[q]; ++e) s_map[base + e] = (uint16_t)s;
            }
            base += my_cnt[q];
        }
        if (threadIdx.x == 0) s_pref[nsrc] = total;
        lds_barrier();
        // the next chunk's ranges load while this chunk deposits
        if (j + 1 < nch) fetch(j + 1);

        for (int e0 = 0; e0 < total; e0 += NT * U) {
            int mm[U][3], src_of[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int e = e0 + u * NT + threadIdx.x;
                src_of[u] = -1;
                if (e < total) {
                    const int s = mapped ? (int)s_map[e] : find_cell_fixed<(MAXSRC <= 256 ? 8 : 10)>(s_pref, nsrc, e);
                    const int pidx = s_start[s] + (e - s_pref[s]);
                    src_of[u] = s;
#pragma unroll
                    for (int k = 0; k < 3; ++k) mm[u][k] = p.m[k][pidx];
                }
            }
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int s = src_of[u];
                if (s < 0) continue;
                const int rl = s_rel[s];
                // coarse cell relative to the column's first cell in x and y
                // and to the chunk's first layer in z
                const int rel[3] = {(rl & 255) - 1, ((rl >> 8) & 255) - 1, rl >> 16};
                int i0[3];
                unsigned w1[3];
#pragma unroll
                for (int k = 0; k < 3; ++k) {
                    const int P = 2 * (rel[k] * 256 + mm[u][k]) + 1;   // units of 1/D target cells
                    const int Pm = P - halfD;
                    i0[k] = Pm >> log2D;                                // floor division
                    w1[k] = (unsigned)(Pm & (D - 1));
                }
#pragma unroll
                for (int oz = 0; oz < 2; ++oz) {
                    // plane i0 + oz of the chunk is accumulator plane i0 + oz + 1, in [0, CZ + 1]
                    const int iz = i0[2] + oz + 1;
                    const unsigned wz = oz ? w1[2] : (unsigned)D - w1[2];
#pragma unroll
                    for (int oy = 0; oy < 2; ++oy) {
                        const int iy = i0[1] + oy;
                        if (iy < 0 || iy >= bwy) continue;
                        const unsigned wyz = (unsigned)__umul24(oy ? w1[1] : (unsigned)D - w1[1], wz);
#pragma unroll
                        for (int ox = 0; ox < 2; ++ox) {
                            const int ix = i0[0] + ox;
                            if (ix < 0 || ix >= bwx) continue;
                            const ACC w = (ACC)(unsigned)__umul24(ox ? w1[0] : (unsigned)D - w1[0], wyz);
                            if (w) atomicAdd(&acc[(iz * BW + iy) * BW + ix], w);
                        }
                    }
                }
            }
        }
        lds_barrier();

        // planes z0 - 1 .. z0 + CZ - 2 are complete (after the last chunk:
        // all of them); four x-consecutive cells per float4 store
        const bool last = j + 1 == nch;
        const int nl = last ? NP : CZ;
        for (int i4 = threadIdx.x; i4 < Q * BW * nl; i4 += NT) {
            const int ix = 4 * (i4 % Q), iy = (i4 / Q) % BW, L = i4 / (Q * BW);
            const int z = j * CZ - 1 + L;
            if (ix >= bwx || iy >= bwy || z < 0 || z >= M) continue;
            const ACC* a = &acc[(L * BW + iy) * BW + ix];
            float4 v;
            if (max(max(a[0], a[1]), max(a[2], a[3])) < (ACC)(1u << 24)) {
                // the sums and the power-of-two scale are exact in FP32, and
                // the fused multiply-add rounds once: the FP64 result
                v.x = fmaf((float)a[0], scalef, -1.0f);
                v.y = fmaf((float)a[1], scalef, -1.0f);
                v.z = fmaf((float)a[2], scalef, -1.0f);
                v.w = fmaf((float)a[3], scalef, -1.0f);
            } else {
                v.x = (float)fma((double)a[0], scale, -1.0);
                v.y = (float)fma((double)a[1], scale, -1.0);
                v.z = (float)fma((double)a[2], scale, -1.0);
                v.w = (float)fma((double)a[3], scale, -1.0);
            }
            const int64_t cell = (int64_t)(T0x + ix) + (int64_t)M * ((T0y + iy) + (int64_t)M * z);
            *reinterpret_cast<float4*>(mesh + cell) = v;
        }
        if (last) break;
        lds_barrier();
        // planes z0 + CZ - 1 and z0 + CZ become the next chunk's first two
        for (int i = threadIdx.x; i < PL; i += NT) {
            const ACC a0 = acc[CZ * PL + i], a1 = acc[(CZ + 1) * PL + i];
            acc[i] = a0;
            acc[PL + i] = a1;
#pragma unroll
            for (int L = 2; L < NP; ++L) acc[L * PL + i] = (ACC)0;
        }
    }
}

// Coarse-mesh deposit (one mesh cell per storage cell): a workgroup owns a
// BW^3 cube of mesh cells and walks the (BW+2)^3 storage cells that can reach
// it, one cell per thread.  Along each axis a particle at in-cell byte m
// weighs (in 1/512 of a cell) 255 - 2m and 2m + 257 on the cells at offsets
// -1 and 0 when m < 128, and 767 - 2m and 2m - 255 on offsets 0 and +1
// otherwise; the thread sums the 27 products over its cell's particles in
// 32-bit registers (each product is below 2^27, so a sum of 24 is exact;
// larger cells are summed 24 particles at a time) and adds each sum that
// lands in the cube to a 64-bit LDS accumulator: one LDS atomic per cell and
// slot instead of eight per particle, and no two lanes of an atomic on one
// address.  The bytes of 8 particles are loaded together and the next cell's
// range is fetched while the current cell is summed.  Integer sums: the
// result does not depend on the order and equals the particle-by-particle
// deposit bit for bit.
template <int BW>
__global__ __launch_bounds__(kDepThreads) void k_coarse_deposit(Geom g, const int32_t* __restrict__ offsets,
                                                                 Planes p, float2* __restrict__ out, double scale) {
    constexpr int SW = BW + 2;
    constexpr int NS = SW * SW * SW;
    constexpr int U = 8;                          // particles whose bytes are in flight together
    constexpr int CH = 3 * U;                     // particles per exact 32-bit partial sum
    __shared__ __align__(16) unsigned long long acc[BW * BW * BW];
    const int M = g.Nc;
    const int nbx = (M + BW - 1) / BW;
    const int b = (int)xcd_logical_block();
    const int T0[3] = {(b % nbx) * BW, ((b / nbx) % nbx) * BW, (b / (nbx * nbx)) * BW};
    const int bw[3] = {min(BW, M - T0[0]), min(BW, M - T0[1]), min(BW, M - T0[2])};
    for (int i = threadIdx.x; i < BW * BW * BW / 2; i += kDepThreads)
        reinterpret_cast<uint4*>(acc)[i] = make_uint4(0u, 0u, 0u, 0u);
    // particle range of window cell s (storage cell T0 - 1 + r); cells past a
    // partial cube's reach are empty
    auto range = [&](int s, int& st, int& en) {
        const int rx = s % SW, ry = (s / SW) % SW, rz = s / (SW * SW);
        st = en = 0;
        if (s < NS && rx <= bw[0] + 1 && ry <= bw[1] + 1 && rz <= bw[2] + 1) {
            const int64_t c = canon(g, wrapi(T0[0] - 1 + rx, M), wrapi(T0[1] - 1 + ry, M), wrapi(T0[2] - 1 + rz, M));
            st = offsets[c];
            en = offsets[c + 1];
        }
    };
    int nst, nen;
    range(threadIdx.x, nst, nen);
    __syncthreads();
    for (int s = threadIdx.x; s < NS; s += kDepThreads) {
        const int st = nst, en = nen;
        range(s + kDepThreads, nst, nen);                         // next cell's range in flight
        const int r[3] = {s % SW, (s / SW) % SW, s / (SW * SW)};
        for (int q0 = st; q0 < en; q0 += CH) {
            const int q1 = min(en, q0 + CH);
            unsigned a[27];
#pragma unroll
            for (int k = 0; k < 27; ++k) a[k] = 0u;
            for (int qb = q0; qb < q1; qb += U) {
                unsigned mm[U][3];
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    const int q = min(qb + u, q1 - 1);
#pragma unroll
                    for (int k = 0; k < 3; ++k) mm[u][k] = p.m[k][q];
                }
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    const bool live = qb + u < q1;
                    unsigned w[3][3];
#pragma unroll
                    for (int k = 0; k < 3; ++k) {
                        const unsigned m = mm[u][k];
                        const bool lo = m < 128u;
                        w[k][0] = lo ? 255u - 2u * m : 0u;
                        w[k][1] = lo ? 2u * m + 257u : 767u - 2u * m;
                        w[k][2] = lo ? 0u : 2u * m - 255u;
                    }
                    if (!live) w[2][0] = w[2][1] = w[2][2] = 0u;
                    unsigned wxy[9];
#pragma unroll
                    for (int j = 0; j < 3; ++j)
#pragma unroll
                        for (int i = 0; i < 3; ++i) wxy[3 * j + i] = (unsigned)__umul24(w[0][i], w[1][j]);
#pragma unroll
                    for (int k = 0; k < 3; ++k)
#pragma unroll
                        for (int j = 0; j < 9; ++j) a[9 * k + j] += (unsigned)__umul24(wxy[j], w[2][k]);
                }
            }
            // slot (i, j, k) lands on cube cell r + (i, j, k) - 2
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                const int tz = r[2] + k - 2;
                if (tz < 0 || tz >= bw[2]) continue;
#pragma unroll
                for (int j = 0; j < 3; ++j) {
                    const int ty = r[1] + j - 2;
                    if (ty < 0 || ty >= bw[1]) continue;
#pragma unroll
                    for (int i = 0; i < 3; ++i) {
                        const int tx = r[0] + i - 2;
                        const unsigned v = a[9 * k + 3 * j + i];
                        if (tx >= 0 && tx < bw[0] && v) atomicAdd(&acc[(tz * BW + ty) * BW + tx], (unsigned long long)v);
                    }
                }
            }
        }
    }
    __syncthreads();
    for (int i = threadIdx.x; i < BW * BW * BW; i += kDepThreads) {
        const int ix = i % BW, iy = (i / BW) % BW, iz = i / (BW * BW);
        if (ix >= bw[0] || iy >= bw[1] || iz >= bw[2]) continue;
        const float v = (float)((double)acc[i] * scale - 1.0);
        out[(int64_t)(T0[0] + ix) + (int64_t)M * ((T0[1] + iy) + (int64_t)M * (T0[2] + iz))] = make_float2(v, 0.0f);
    }
}

// largest particle count of any 2 x 2 x 2 block of coarse cells (periodic).
// Cells are visited in storage order (the +x, +y, +z neighbours are then
// mostly 1, Tc and Tc^2 entries ahead); one atomic per workgroup.
__global__ __launch_bounds__(256) void k_max_block8(Geom g, const int32_t* __restrict__ counts,
                                                      int32_t* __restrict__ out, const int32_t* gate) {
    if (gate && *(volatile const int32_t*)gate) return;
    __shared__ int red[256 / kWave];
    const int64_t tc3 = (int64_t)g.Tc * g.Tc * g.Tc;
    int v = 0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < g.ncells;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t tile = i / tc3;
        const int local = (int)(i - tile * tc3);
        const int tx = (int)(tile % g.nt), ty = (int)((tile / g.nt) % g.nt), tz = (int)(tile / ((int64_t)g.nt * g.nt));
        const int cx = tx * g.Tc + local % g.Tc, cy = ty * g.Tc + (local / g.Tc) % g.Tc;
        const int cz = tz * g.Tc + local / (g.Tc * g.Tc);
        const int x1 = cx + 1 == g.Nc ? 0 : cx + 1, y1 = cy + 1 == g.Nc ? 0 : cy + 1;
        const int z1 = cz + 1 == g.Nc ? 0 : cz + 1;
        const int sum = counts[i] + counts[canon(g, x1, cy, cz)] + counts[canon(g, cx, y1, cz)] +
                        counts[canon(g, x1, y1, cz)] + counts[canon(g, cx, cy, z1)] + counts[canon(g, x1, cy, z1)] +
                        counts[canon(g, cx, y1, z1)] + counts[canon(g, x1, y1, z1)];
        v = max(v, sum);
    }
    v = wave_max(v);
    if ((threadIdx.x & (kWave - 1)) == 0) red[threadIdx.x / kWave] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < 256 / kWave; ++w) v = max(v, red[w]);
        atomicMax(out, v);
    }
}

int ilog2(int v) {
    int l = 0;
    while ((1 << l) < v) ++l;
    return l;
}

}  // namespace

void launch_coarse_deposit(const Geom& g, const int32_t* offsets, Planes p, float2* mesh, int32_t* /*overflow*/,
                           hipStream_t s) {
    constexpr int BW = 16;
    const int nb = (g.Nc + BW - 1) / BW;
    // acc in units of 2^-27 particle; density = mass / H^3 with H = r / f
    const double scale = std::ldexp(1.0, -27) * ((double)g.f * g.f * g.f) / ((double)g.r * g.r * g.r);
    hipLaunchKernelGGL((k_coarse_deposit<BW>), dim3(nb * nb * nb), dim3(kDepThreads), 0, s, g, offsets, p, mesh,
                       scale);
}

void launch_fine_deposit(const Geom& g, const int32_t* offsets, Planes p, int tile0, int ntiles,
                         float* mesh, bool wide, hipStream_t s) {
    // every box has r = 4 or r = 8 (the gather's bricks need it)
    const int log2D = g.log2D;
    // acc in units of D^-3 fine-cell masses; density = mass / h^3 = mass * f^3
    const double scale = std::ldexp(1.0, -3 * log2D) * ((double)g.f * g.f * g.f);
    if (g.periodic) {
        // the single periodic tile: 16^3 bricks over (16 / r + 2)^3 <= 6^3 source cells
        const int nb = (g.F + 15) / 16;
        const dim3 grid(nb * nb * nb, ntiles), block(kDepThreads);
        if (wide)
            hipLaunchKernelGGL((k_deposit<16, DEP_FINE_PERIODIC, unsigned long long, 216, 2048>), grid, block, 0, s,
                               g, offsets, p, mesh, g.F, g.r, log2D, scale, tile0);
        else
            hipLaunchKernelGGL((k_deposit<16, DEP_FINE_PERIODIC, unsigned int, 216, 2048>), grid, block, 0, s, g,
                               offsets, p, mesh, g.F, g.r, log2D, scale, tile0);
        return;
    }
    // tile meshes:
    // z-marching columns of 32 x 32 cells in chunks of 8 planes on 512
    // threads, 4 particles in flight per thread -- the fastest shape measured
    // at 1024^3 (10 x 10 x 2 source cells per chunk for r = 4, 6 x 6 x 1 for
    // r = 8)
    const int nbz = (g.F + 31) / 32;
    if (wide)
        hipLaunchKernelGGL((k_deposit_zm<32, 8, 512, 4, unsigned long long, 200, 4096>), dim3(nbz * nbz, ntiles),
                           dim3(512), 0, s, g, offsets, p, mesh, g.r, log2D, scale, tile0);
    else
        hipLaunchKernelGGL((k_deposit_zm<32, 8, 512, 4, unsigned int, 200, 4096>), dim3(nbz * nbz, ntiles),
                           dim3(512), 0, s, g, offsets, p, mesh, g.r, log2D, scale, tile0);
}

bool fine_deposit_needs_wide(const Geom& g, int max_block8) {
    // a fine cell gathers the particles of at most one 2 x 2 x 2 block of
    // coarse cells, each weighing at most D^3 units: stay below 2^32
    return (double)max_block8 * std::ldexp(1.0, 3 * g.log2D) >= 4294967296.0;
}

bool fp16_density_fits(const Geom& g, int max_block8) {
    // a fine cell's density is at most f^3 times the particles of one 2 x 2 x 2
    // block of coarse cells; the plane transform's gain is divided out
    return (double)g.f * g.f * g.f * (double)max_block8 + 1.0 < 32768.0;
}

void launch_max_block8(const Geom& g, const int32_t* counts, int32_t* out, hipStream_t s, const int32_t* gate) {
    const int64_t want = (g.ncells + 255) / 256;
    hipLaunchKernelGGL(k_max_block8, dim3((unsigned)std::min<int64_t>(want, 4096)), dim3(256), 0, s, g, counts, out,
                       gate);
}

void launch_diag_deposit(const Geom& g, const int32_t* offsets, Planes p, float2* mesh, hipStream_t s) {
    constexpr int BW = 8;
    const int H = g.r / g.f;                       // diagnostic cells per coarse cell
    const int nb = (g.ns + BW - 1) / BW;
    const int log2D = ilog2(512 / H);
    const double scale = std::ldexp(1.0, -3 * log2D);
    hipLaunchKernelGGL((k_deposit<BW, DEP_DIAG, unsigned long long, 1000, 10240>), dim3(nb * nb * nb),
                       dim3(kDepThreads), 0, s, g, offsets, p, reinterpret_cast<float*>(mesh), g.ns, H, log2D,
                       scale, 0);
}

}  // namespace cube
