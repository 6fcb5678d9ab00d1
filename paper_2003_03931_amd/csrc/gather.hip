// Force interpolation, kick, drift and recount (Sec. II: the PM force is the
// long-range coarse-mesh part plus the short-range part of the particle's own
// tile; Sec. III-A: positions and velocities are re-encoded after the update).
//
// One workgroup per brick of 32 x 16 x 8 fine cells of one tile.  It stages
// the tile's fine potential over the brick plus a halo of H cells and the
// coarse potential over the brick's coarse cells plus H cells in LDS (H = 2
// for 2-point differences, 3 for 4-point ones: the CIC nodes reach one cell
// out, the difference stencil H - 1 more), then walks the brick's particles
// (its coarse cells' contiguous ranges):
//   * decode (Eq. (2)) into fine and coarse coordinates, exactly;
//   * a = CIC-gather of -grad phi_f + CIC-gather of -grad phi_c, gradients by
//     2- or 4-point central differences taken on the fly from the LDS
//     potentials;
//   * kick in FP64:  u' = clamp(rint((u s + a K) / s'), -127, 127);
//   * drift in cell-local quanta, exactly in FP64:
//       X = m + 1/2 + ((u' s') (256/H)) D,  q = floor(X),
//       carry = floor(q / 256), m' = q mod 256, cell' = cell + carry (periodic);
//   * write (m', u') at the same index of the second particle buffer and a
//     move code for the compaction; new-cell counts go to an LDS histogram
//     over the brick's cells plus one cell, flushed once per brick.
// K and D are the step's kick and drift multipliers: dt and dt in a static
// box, the comoving integrals (D rounded to FP32) in an expanding one.
#include <type_traits>

#include "common.h"

namespace cube {

namespace {

constexpr int kBX = kGBX, kBY = kGBY, kBZ = kGBZ;       // brick, fine cells
constexpr int kMinR = 4;                                 // coarse cells of >= 4 fine cells
constexpr int kMaxRows = (kBY / kMinR) * (kBZ / kMinR);
constexpr int kMaxRowLen = kBX / kMinR;
static_assert(kMaxRows <= 8 && kMaxRowLen <= 8, "fixed three-step searches of rows and cells");
constexpr int kMaxHist = (kBX / kMinR + 2) * (kBY / kMinR + 2) * (kBZ / kMinR + 2);
constexpr int kGatherThreads = 256;
constexpr int kGatherMovCap = 480;                       // movers of a brick listed in LDS

// extents of the staged potentials for a halo of H cells
template <int H>
struct Halo {
    static constexpr int LX = kBX + 2 * H, LY = kBY + 2 * H, LZ = kBZ + 2 * H;
    static constexpr int COARSE = (kBX / kMinR + 2 * H) * (kBY / kMinR + 2 * H) * (kBZ / kMinR + 2 * H);
};

// class 0..26 of the brick that a brick-relative cell (x, y, z), each in
// [-1, extent], lies in: (dx + 1) + 3 (dy + 1) + 9 (dz + 1), 13 = this brick
__device__ __forceinline__ int move_class(int x, int y, int z, int bx, int by, int bz) {
    const int dx = x < 0 ? -1 : (x >= bx ? 1 : 0), dy = y < 0 ? -1 : (y >= by ? 1 : 0);
    const int dz = z < 0 ? -1 : (z >= bz ? 1 : 0);
    return (dx + 1) + 3 * (dy + 1) + 9 * (dz + 1);
}

struct LdsGrid {
    const float* p;
    int sx, sxy;      // strides
    __device__ float at(int x, int y, int z) const { return p[(z * sxy) + y * sx + x]; }
};

// w0 (-D phi)(i0) + w1 (-D phi)(i0 + 1) from v[j] = phi(i0 - R + j), without
// the 1/(2h) or 1/(12h) factor: D phi(n) = phi(n+1) - phi(n-1) for R = 1,
// 8 (phi(n+1) - phi(n-1)) - (phi(n+2) - phi(n-2)) for R = 2.
template <int R>
__device__ __forceinline__ float neg_diff_interp(const float* v, float w0, float w1) {
    if constexpr (R == 1)
        return w0 * (v[0] - v[2]) + w1 * (v[1] - v[3]);
    else
        return w0 * (8.0f * (v[1] - v[3]) - (v[0] - v[4])) + w1 * (8.0f * (v[2] - v[4]) - (v[1] - v[5]));
}

// CIC gather of -grad(phi) with a difference stencil of reach R: i0/t per
// axis in LDS-grid coordinates, `scale` the difference's 1/(2h) or 1/(12h).
template <int R>
__device__ __forceinline__ void gather_force(const LdsGrid& phi, const int i0[3], const float t[3], float scale,
                                             float out[3]) {
    const float w[3][2] = {{1.0f - t[0], t[0]}, {1.0f - t[1], t[1]}, {1.0f - t[2], t[2]}};
    float ax = 0.f, ay = 0.f, az = 0.f;
    float v[2 * R + 2];
#pragma unroll
    for (int oz = 0; oz < 2; ++oz)
#pragma unroll
        for (int oy = 0; oy < 2; ++oy) {
            const int y = i0[1] + oy, z = i0[2] + oz;
#pragma unroll
            for (int j = 0; j < 2 * R + 2; ++j) v[j] = phi.at(i0[0] - R + j, y, z);
            ax += w[1][oy] * w[2][oz] * neg_diff_interp<R>(v, w[0][0], w[0][1]);
        }
#pragma unroll
    for (int oz = 0; oz < 2; ++oz)
#pragma unroll
        for (int ox = 0; ox < 2; ++ox) {
            const int x = i0[0] + ox, z = i0[2] + oz;
#pragma unroll
            for (int j = 0; j < 2 * R + 2; ++j) v[j] = phi.at(x, i0[1] - R + j, z);
            ay += w[0][ox] * w[2][oz] * neg_diff_interp<R>(v, w[1][0], w[1][1]);
        }
#pragma unroll
    for (int oy = 0; oy < 2; ++oy)
#pragma unroll
        for (int ox = 0; ox < 2; ++ox) {
            const int x = i0[0] + ox, y = i0[1] + oy;
#pragma unroll
            for (int j = 0; j < 2 * R + 2; ++j) v[j] = phi.at(x, y, i0[2] - R + j);
            az += w[0][ox] * w[1][oy] * neg_diff_interp<R>(v, w[2][0], w[2][1]);
        }
    out[0] = ax * scale;
    out[1] = ay * scale;
    out[2] = az * scale;
}

__device__ __forceinline__ float gather_value(const LdsGrid& phi, const int i0[3], const float t[3]) {
    float acc = 0.f;
#pragma unroll
    for (int oz = 0; oz < 2; ++oz)
#pragma unroll
        for (int oy = 0; oy < 2; ++oy)
#pragma unroll
            for (int ox = 0; ox < 2; ++ox)
                acc += (ox ? t[0] : 1.f - t[0]) * (oy ? t[1] : 1.f - t[1]) * (oz ? t[2] : 1.f - t[2]) *
                       phi.at(i0[0] + ox, i0[1] + oy, i0[2] + oz);
    return acc;
}

// PER: the single periodic tile (the fine halo wraps, staged one float at a
// time); otherwise every staged row is read as aligned float2s.  The row's
// first wanted float has the parity of H (the buffer and the brick origin
// are even), so odd H stages one extra float on the left and possibly one
// past the row's end (the mesh allocation is padded for the last row).
// VC (step mode only): velocities in the cell-mean codec (Eq. (3)); the
// kicked velocity is written to the FP32 working planes instead of codes.
template <int MODE, int H, bool PER, bool VC = false, int RC = 0>
__global__ __launch_bounds__(kGatherThreads) void k_gather(GatherArgs A) {
    constexpr int kLX = Halo<H>::LX, kLY = Halo<H>::LY, kLZ = Halo<H>::LZ;
    constexpr int kSlack = H & 1;                  // floats staged before the wanted ones
    constexpr int kRow2 = (kLX + kSlack + 1) / 2;  // float2 per staged row
    constexpr int kSX = 2 * kRow2;                 // LDS row stride, floats
    constexpr int kFineLds = kSX * kLY * kLZ, kMaxCoarseLds = Halo<H>::COARSE;
    __shared__ __align__(8) float s_fine[kFineLds];
    __shared__ float s_coarse[kMaxCoarseLds];
    __shared__ int s_rowoff[kMaxRows][kMaxRowLen + 1];
    __shared__ int s_rowpref[kMaxRows + 1];
    __shared__ int s_hist[kMaxHist];
    __shared__ int s_scan[kGatherThreads / kWave + 1];
    __shared__ double s_red[kGatherThreads / kWave];
    __shared__ float s_vc[3][VC ? kMaxRows * kMaxRowLen : 1];   // cell means of the brick's cells
    __shared__ int s_ccount[28], s_crun[27];                    // movers per destination-brick class
    __shared__ int s_hist_base;
    __shared__ int s_nmov, s_mov[MODE == GATHER_STEP ? kGatherMovCap : 1];   // the brick's movers, if they fit

    // a halted step (see StepScalars) writes nothing
    if (MODE == GATHER_STEP && *(volatile const int32_t*)&A.sc->halt) return;
    const Geom& g = A.g;
    // RC: fine cells per coarse cell fixed at compile time (0: read from g),
    // which turns the brick's cell-index divisions into shifts
    const int r = RC ? RC : g.r;
    const int BXc = kBX / r, BYc = kBY / r, BZc = kBZ / r;
    const int nrows = BYc * BZc;
    const int64_t lb = xcd_logical_block();
    const int k = (int)(lb / gridDim.x);                   // tile within the batch
    const int tile = A.tile0 + k;
    const int nbx = g.T / kBX, nby = g.T / kBY;
    const int b = (int)(lb % gridDim.x);
    const int bx = b % nbx, by = (b / nbx) % nby, bz = b / (nbx * nby);
    const int tx = tile % g.nt, ty = (tile / g.nt) % g.nt, tz = tile / (g.nt * g.nt);
    // brick origin: tile-local fine and coarse coordinates, global coarse
    const int lf[3] = {bx * kBX, by * kBY, bz * kBZ};
    const int lc[3] = {lf[0] / r, lf[1] / r, lf[2] / r};
    const int gc[3] = {tx * g.Tc + lc[0], ty * g.Tc + lc[1], tz * g.Tc + lc[2]};

    // fine potential of the brick plus H cells: tile-box coords b + lf - H ...
    const float* fmesh = A.fine_real + (int64_t)k * g.F * g.F * g.F;   // tile k of the batch
    const int F = g.F, ox = g.b + lf[0] - H, oy = g.b + lf[1] - H, oz = g.b + lf[2] - H;
    // Every load of the staging phase (fine potential with halo, coarse
    // potential with halo, row offsets) is issued before the first wait: one
    // memory latency per block instead of one per round.
    const int CX = BXc + 2 * H, CY = BYc + 2 * H, CZ = BZc + 2 * H;
    // the coarse grid is laid out with the strides of the largest brick
    // (r = kMinR), constants the LDS reads fold into their offsets
    constexpr int kCSX = kBX / kMinR + 2 * H, kCSXY = kCSX * (kBY / kMinR + 2 * H);
    const float* cmesh = reinterpret_cast<const float*>(A.coarse);
    const int Nc = g.Nc, cx0 = gc[0] - H, cy0 = gc[1] - H, cz0 = gc[2] - H;
    const int ncoarse = CX * CY * CZ, nrowoff = nrows * (BXc + 1);
    constexpr int NS = kLX * kLY * kLZ;            // periodic: scalar elements
    constexpr int NV = kRow2 * kLY * kLZ;          // tiled: float2 elements
    constexpr int UF = ((PER ? NS : NV) + kGatherThreads - 1) / kGatherThreads;
    constexpr int UC = (kMaxCoarseLds + kGatherThreads - 1) / kGatherThreads;
    constexpr int UR = (kMaxRows * (kMaxRowLen + 1) + kGatherThreads - 1) / kGatherThreads;
    typedef float f2 __attribute__((ext_vector_type(2)));
    using FV = typename std::conditional<PER, float, f2>::type;
    FV fv[UF];
    float cv[UC];
    int cl[UC];
    int rv[UR];
    const int ox_al = ox - kSlack;                 // even
    const int a_off = PER ? 0 : kSlack;            // first wanted float within the staged row
#pragma unroll
    for (int u = 0; u < UF; ++u) {
        const int e = threadIdx.x + u * kGatherThreads;
        if constexpr (PER) {
            if (e < NS) {
                int fx = ox + e % kLX, fy = oy + (e / kLX) % kLY, fz = oz + e / (kLX * kLY);
                fx = fx < 0 ? fx + F : (fx >= F ? fx - F : fx);
                fy = fy < 0 ? fy + F : (fy >= F ? fy - F : fy);
                fz = fz < 0 ? fz + F : (fz >= F ? fz - F : fz);
                fv[u] = fmesh[(fz * F + fy) * F + fx];
            }
        } else {
            if (e < NV) {
                const int x2 = e % kRow2, row = e / kRow2, y = row % kLY, z = row / kLY;
                fv[u] = *reinterpret_cast<const f2*>(fmesh + ((oz + z) * F + (oy + y)) * F + ox_al + 2 * x2);
            }
        }
    }
    // window coordinates by float reciprocals (exact: e < 2^11, extents <= 2^8)
    const float inv_cx = 1.0f / (float)CX, inv_cxy = 1.0f / (float)(CX * CY);
#pragma unroll
    for (int u = 0; u < UC; ++u) {
        const int e = threadIdx.x + u * kGatherThreads;
        if (e < ncoarse) {
            const int ez = (int)(((float)e + 0.5f) * inv_cxy), rem = e - ez * (CX * CY);
            const int ey = (int)(((float)rem + 0.5f) * inv_cx), ex = rem - ey * CX;
            cl[u] = ez * kCSXY + ey * kCSX + ex;
            int cx = cx0 + ex, cy = cy0 + ey, cz = cz0 + ez;
            cx = cx < 0 ? cx + Nc : (cx >= Nc ? cx - Nc : cx);
            cy = cy < 0 ? cy + Nc : (cy >= Nc ? cy - Nc : cy);
            cz = cz < 0 ? cz + Nc : (cz >= Nc ? cz - Nc : cz);
            cv[u] = cmesh[2 * (((int64_t)cz * Nc + cy) * Nc + cx)];
        }
    }
#pragma unroll
    for (int u = 0; u < UR; ++u) {
        const int e = threadIdx.x + u * kGatherThreads;
        if (e < nrowoff) {
            const int row = e / (BXc + 1), j = e % (BXc + 1);
            const int ry = row % BYc, rz = row / BYc;
            rv[u] = A.offsets[canon(g, gc[0], gc[1] + ry, gc[2] + rz) + j];
        }
    }
#pragma unroll
    for (int u = 0; u < UF; ++u) {
        const int e = threadIdx.x + u * kGatherThreads;
        if constexpr (PER) {
            if (e < NS) s_fine[((e / (kLX * kLY)) * kLY + (e / kLX) % kLY) * kSX + e % kLX] = fv[u];
        } else {
            if (e < NV) reinterpret_cast<f2*>(s_fine)[e] = fv[u];
        }
    }
#pragma unroll
    for (int u = 0; u < UC; ++u) {
        const int e = threadIdx.x + u * kGatherThreads;
        if (e < ncoarse) s_coarse[cl[u]] = cv[u];
    }
#pragma unroll
    for (int u = 0; u < UR; ++u) {
        const int e = threadIdx.x + u * kGatherThreads;
        if (e < nrowoff) s_rowoff[e / (BXc + 1)][e % (BXc + 1)] = rv[u];
    }
    const int HX = BXc + 2, HY = BYc + 2, HZ = BZc + 2;
    if (MODE == GATHER_STEP) {
        for (int e = threadIdx.x; e < HX * HY * HZ; e += kGatherThreads) s_hist[e] = 0;
        if ((int)threadIdx.x < 28) s_ccount[threadIdx.x] = 0;
        if (threadIdx.x == 0) s_nmov = 0;
        if ((int)threadIdx.x < 27) s_crun[threadIdx.x] = 0;
    }
    if constexpr (VC) {
        const int nbc = BXc * BYc * BZc;
        for (int e = threadIdx.x; e < 3 * nbc; e += kGatherThreads) {
            const int k3 = e / nbc, cl = e - k3 * nbc;
            const int lx = cl % BXc, ly = (cl / BXc) % BYc, lz = cl / (BXc * BYc);
            s_vc[k3][cl] = A.vcell.vc[k3][canon(g, gc[0] + lx, gc[1] + ly, gc[2] + lz)];
        }
    }
    __syncthreads();
    {
        const int row = threadIdx.x;
        const int cnt = row < nrows ? s_rowoff[row][BXc] - s_rowoff[row][0] : 0;
        int total;
        const int pref = block_exclusive_scan(cnt, s_scan, &total);
        if (row < nrows) s_rowpref[row] = pref;
        if (row == 0) s_rowpref[nrows] = total;
    }
    __syncthreads();

    const LdsGrid fphi{s_fine + a_off, kSX, kSX * kLY};
    const LdsGrid cphi{s_coarse, kCSX, kCSXY};
    const int D = 1 << g.log2D, halfD = D >> 1;
    const float invD = 1.0f / (float)D;
    constexpr int R = H - 1;                                 // difference reach
    // 1 / (2h) and 1 / (2H), or 1 / (12h) and 1 / (12H)
    const float scale_f = R == 1 ? (float)g.f * 0.5f : (float)g.f / 12.0f;
    const float scale_c = R == 1 ? (float)g.f / (2.0f * (float)r) : (float)g.f / (12.0f * (float)r);
    double s = 0.0, s_next = 0.0, inv_s_next = 0.0;
    if (MODE == GATHER_STEP) {
        s = A.sc->s;
        s_next = A.sc->s_next;
        inv_s_next = 1.0 / s_next;                           // exact: s' is a power of two
    }
    const double q256H = 256.0 * g.f / r;                    // 256 / H
    const double kick = A.kick, drift = (double)A.drift;

    int umax = 0, sat = 0, cmax = 0, nfar = 0;
    double esum = 0.0;
    const int total = s_rowpref[nrows];
    // the brick's slots in its tile's region of the mover-record array: one
    // per particle, reserved now so the atomic's latency hides behind the loop
    int rbase = 0;
    if (MODE == GATHER_STEP && threadIdx.x == 0 && total > 0) rbase = atomicAdd(&A.tcursor[tile], total);
    // software pipeline: the next particle's bytes are in flight while the
    // current one is computed
    auto locate = [&](int e, int& p, int& lx, int& ly, int& lz) {
        const int row = find_cell_fixed<3>(s_rowpref, nrows, e);      // nrows <= 8
        p = s_rowoff[row][0] + (e - s_rowpref[row]);
        lx = find_cell_fixed<3>(s_rowoff[row], BXc, p);              // BXc <= 8
        ly = row % BYc;
        lz = row / BYc;
    };
    int np_ = 0, nlx = 0, nly = 0, nlz = 0, nm[3] = {0, 0, 0}, nu[3] = {0, 0, 0};
    if ((int)threadIdx.x < total) {
        locate(threadIdx.x, np_, nlx, nly, nlz);
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            nm[a] = A.in.m[a][(uint32_t)np_];
            if (MODE == GATHER_STEP) nu[a] = A.in.u[a][(uint32_t)np_];
        }
    }
    for (int e = threadIdx.x; e < total; e += kGatherThreads) {
        const int p = np_;
        const int lcell[3] = {nlx, nly, nlz};                // cell within the brick
        int m[3], uo[3];
#pragma unroll
        for (int a = 0; a < 3; ++a) { m[a] = nm[a]; uo[a] = nu[a]; }
        if (e + kGatherThreads < total) {
            locate(e + kGatherThreads, np_, nlx, nly, nlz);
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                nm[a] = A.in.m[a][(uint32_t)np_];
                if (MODE == GATHER_STEP) nu[a] = A.in.u[a][(uint32_t)np_];
            }
        }
        int fi[3], ci[3];
        float ft[3], ct[3];
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            // fine: brick-relative position in 1/D cells, LDS origin at -H
            const int Pf = 2 * (lcell[a] * 256 + m[a]) + 1 - halfD;
            fi[a] = (Pf >> g.log2D) + H;
            ft[a] = (float)(Pf & (D - 1)) * invD;
            // coarse: brick-relative in 1/512 coarse cells, LDS origin at -H
            const int Pc = 2 * (lcell[a] * 256 + m[a]) + 1 - 256;
            ci[a] = (Pc >> 9) + H;
            ct[a] = (float)(Pc & 511) * (1.0f / 512.0f);
        }
        if (MODE == GATHER_POTENTIAL) {
            esum += (double)gather_value(fphi, fi, ft) + (double)gather_value(cphi, ci, ct);
            continue;
        }
        float af[3], ac[3];
        gather_force<R>(fphi, fi, ft, scale_f, af);
        gather_force<R>(cphi, ci, ct, scale_c, ac);
        float acc[3] = {af[0] + ac[0], af[1] + ac[1], af[2] + ac[2]};
        if (A.pp[0]) {
#pragma unroll
            for (int a = 0; a < 3; ++a) acc[a] += A.pp[a][p];
        }
        if (MODE == GATHER_FORCE) {
#pragma unroll
            for (int a = 0; a < 3; ++a) A.acc[3 * (int64_t)p + a] = acc[a];
            continue;
        }
        int un[3] = {0, 0, 0}, carry[3], mnew[3];
        if constexpr (VC) {
            // decode v_c + sigma tan(u pi / 255), kick in FP64 (one rounding per
            // operation), hold in FP32, drift by it (exact FP64)
            const int cl = (lcell[2] * BYc + lcell[1]) * BXc + lcell[0];
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                const double v = vc_decode(s_vc[a][cl], s, A.vcell.tab, uo[a]);
                const float v32 = (float)__dadd_rn(v, __dmul_rn((double)acc[a], kick));
                A.out.v[a][p] = v32;
                const double X = ((double)m[a] + 0.5) + ((double)v32 * q256H) * drift;
                const int qq = (int)floor(X);
                carry[a] = qq >> 8;
                mnew[a] = qq & 255;
                A.out.m[a][(uint32_t)p] = (uint8_t)mnew[a];
                cmax = max(cmax, abs(carry[a]));
            }
        } else {
        // kick (FP64) and requantise; drift in cell-local quanta (exact FP64)
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            const double v = (double)uo[a] * s + (double)acc[a] * kick;
            double w = rint(v * inv_s_next);
            sat += fabs(w) > 127.0;
            w = fmin(fmax(w, -127.0), 127.0);
            un[a] = (int)w;
            umax = max(umax, abs(un[a]));
            const double X = ((double)m[a] + 0.5) + (((double)un[a] * s_next) * q256H) * drift;
            const int qq = (int)floor(X);
            carry[a] = qq >> 8;                  // floor division by 256
            mnew[a] = qq & 255;
            A.out.m[a][(uint32_t)p] = (uint8_t)mnew[a];
            A.out.u[a][(uint32_t)p] = (int8_t)un[a];
            cmax = max(cmax, abs(carry[a]));
        }
        }
        if (A.out.ids) A.out.ids[p] = A.in.ids[p];
        const bool near = abs(carry[0]) <= 1 && abs(carry[1]) <= 1 && abs(carry[2]) <= 1;
        if (near) {
            const int code = (carry[0] + 1) + 3 * (carry[1] + 1) + 9 * (carry[2] + 1);
            A.dir[(uint32_t)p] = (uint8_t)code;
            const int hx = lcell[0] + carry[0] + 1, hy = lcell[1] + carry[1] + 1, hz = lcell[2] + carry[2] + 1;
            atomicAdd(&s_hist[(hz * HY + hy) * HX + hx], 1);
            if (code != 13) {
                atomicAdd(&s_ccount[move_class(hx - 1, hy - 1, hz - 1, BXc, BYc, BZc)], 1);
                const int k = atomicAdd(&s_nmov, 1);
                if (k < kGatherMovCap) s_mov[k] = p;
            }
        } else {
            const int64_t cn = canon(g, wrapi(gc[0] + lcell[0] + carry[0], g.Nc),
                                     wrapi(gc[1] + lcell[1] + carry[1], g.Nc),
                                     wrapi(gc[2] + lcell[2] + carry[2], g.Nc));
            A.dir[p] = 255;
            A.far_key[p] = (uint32_t)cn;
            atomicAdd(&A.counts_new[cn], 1);
            ++nfar;
        }
    }

    if (MODE == GATHER_STEP) {
        __syncthreads();
        // Mover records, grouped by the class of their destination brick, in
        // the brick's reserved slots: the movers listed in LDS (or, too many,
        // all particles again) with the codes and bytes just written.
        if (threadIdx.x < kWave) {
            const int lane = threadIdx.x;
            const int v = lane < 27 ? s_ccount[lane] : 0;
            const int incl = wave_inclusive_scan(v);
            int32_t* h = A.mhdr + ((int64_t)tile * gridDim.x + b) * kHdrInts;
            if (lane < 27) {
                s_ccount[lane] = incl - v;
                h[1 + lane] = incl - v;
            }
            if (lane == 26) {
                s_ccount[27] = incl;
                h[28] = incl;
            }
            if (lane == 0) {
                h[0] = rbase;
                s_hist_base = rbase;
            }
        }
        __syncthreads();
        if (s_ccount[27] > 0) {
            const int rslot = s_hist_base;
            // the listed movers, or (too many to list) every particle again
            const bool listed = s_nmov <= kGatherMovCap;
            const int nwalk = listed ? s_nmov : total;
            for (int e = threadIdx.x; e < nwalk; e += kGatherThreads) {
                int p, lx, ly, lz;
                if (listed) {
                    p = s_mov[e];
                    int row = 0;                   // the last row starting at or before p
                    for (int r2 = 1; r2 < nrows; ++r2) row = s_rowoff[r2][0] <= p ? r2 : row;
                    lx = find_cell_fixed<3>(s_rowoff[row], BXc, p);
                    ly = row % BYc;
                    lz = row / BYc;
                } else {
                    locate(e, p, lx, ly, lz);
                }
                const int code = A.dir[(uint32_t)p];
                if (code == 13 || code >= 27) continue;
                const int nx = lx + code % 3 - 1, ny = ly + (code / 3) % 3 - 1, nz = lz + code / 9 - 1;
                const int cls = move_class(nx, ny, nz, BXc, BYc, BZc);
                const int bdx = cls % 3 - 1, bdy = (cls / 3) % 3 - 1, bdz = cls / 9 - 1;
                const int dl = (nx - bdx * BXc) + BXc * ((ny - bdy * BYc) + BYc * (nz - bdz * BZc));
                uint4 rec;
                rec.x = (uint32_t)p;
                rec.y = (uint32_t)dl | ((uint32_t)cls << 8);
                rec.z = (uint32_t)A.out.m[0][(uint32_t)p] | ((uint32_t)A.out.m[1][(uint32_t)p] << 8) | ((uint32_t)A.out.m[2][(uint32_t)p] << 16);
                rec.w = 0;
                if constexpr (!VC)
                    rec.w = (uint32_t)(uint8_t)A.out.u[0][(uint32_t)p] | ((uint32_t)(uint8_t)A.out.u[1][(uint32_t)p] << 8) |
                            ((uint32_t)(uint8_t)A.out.u[2][(uint32_t)p] << 16);
                A.ment[rslot + s_ccount[cls] + atomicAdd(&s_crun[cls], 1)] = rec;
            }
        }
        for (int e = threadIdx.x; e < HX * HY * HZ; e += kGatherThreads) {
            const int c = s_hist[e];
            if (c) {
                const int hx = e % HX, hy = (e / HX) % HY, hz = e / (HX * HY);
                int cx = gc[0] + hx - 1, cy = gc[1] + hy - 1, cz = gc[2] + hz - 1;
                cx = cx < 0 ? cx + g.Nc : (cx >= g.Nc ? cx - g.Nc : cx);
                cy = cy < 0 ? cy + g.Nc : (cy >= g.Nc ? cy - g.Nc : cy);
                cz = cz < 0 ? cz + g.Nc : (cz >= g.Nc ? cz - g.Nc : cz);
                const int64_t cn = canon(g, cx, cy, cz);
                atomicAdd(&A.counts_new[cn], c);
            }
        }
        // block reduction, then one atomic per block into one of 64 slots
        __shared__ int s_r[4][kGatherThreads / kWave];
        umax = wave_max(umax);
        cmax = wave_max(cmax);
        sat = wave_sum(sat);
        nfar = wave_sum(nfar);
        if ((threadIdx.x & (kWave - 1)) == 0) {
            const int w = threadIdx.x / kWave;
            s_r[0][w] = umax;
            s_r[1][w] = cmax;
            s_r[2][w] = sat;
            s_r[3][w] = nfar;
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            int bu = 0, bc = 0, bs = 0, bf = 0;
            for (int w = 0; w < kGatherThreads / kWave; ++w) {
                bu = max(bu, s_r[0][w]);
                bc = max(bc, s_r[1][w]);
                bs += s_r[2][w];
                bf += s_r[3][w];
            }
            const int slot = (blockIdx.x + blockIdx.y * 7) & 63;
            if (bu) atomicMax(&A.sc->umax_slot[slot], bu);
            if (bc) atomicMax(&A.sc->cmax_slot[slot], bc);
            if (bs) atomicAdd((unsigned long long*)&A.sc->sat_step, (unsigned long long)bs);
            if (bf) atomicAdd(&A.sc->far_count, bf);
        }
    } else if (MODE == GATHER_POTENTIAL) {
        esum = wave_sum_d(esum);
        if ((threadIdx.x & (kWave - 1)) == 0) s_red[threadIdx.x / kWave] = esum;
        __syncthreads();
        if (threadIdx.x == 0) {
            double t = 0.0;
            for (int w = 0; w < kGatherThreads / kWave; ++w) t += s_red[w];
            A.partial[(int64_t)k * gridDim.x + b] = t;
        }
    }
}

}  // namespace

int gather_blocks_per_tile(const Geom& g) { return (g.T / kBX) * (g.T / kBY) * (g.T / kBZ); }

bool gather_supported(const Geom& g) {
    return g.T % kBX == 0 && g.T % kBY == 0 && g.r >= kMinR && kBZ % g.r == 0;
}

template <int H, bool PER, bool VC>
void launch_gather_step(const GatherArgs& a, const dim3& grid, hipStream_t s) {
    if (a.g.r == 4)
        hipLaunchKernelGGL((k_gather<GATHER_STEP, H, PER, VC, 4>), grid, dim3(kGatherThreads), 0, s, a);
    else if (a.g.r == 8)
        hipLaunchKernelGGL((k_gather<GATHER_STEP, H, PER, VC, 8>), grid, dim3(kGatherThreads), 0, s, a);
    else
        hipLaunchKernelGGL((k_gather<GATHER_STEP, H, PER, VC>), grid, dim3(kGatherThreads), 0, s, a);
}

template <int H, bool PER>
void launch_gather_halo(const GatherArgs& a, const dim3& grid, hipStream_t s) {
    if (a.mode == GATHER_STEP && a.g.vcodec)
        launch_gather_step<H, PER, true>(a, grid, s);
    else if (a.mode == GATHER_STEP)
        launch_gather_step<H, PER, false>(a, grid, s);
    else if (a.mode == GATHER_FORCE)
        hipLaunchKernelGGL((k_gather<GATHER_FORCE, H, PER>), grid, dim3(kGatherThreads), 0, s, a);
    else
        hipLaunchKernelGGL((k_gather<GATHER_POTENTIAL, H, PER>), grid, dim3(kGatherThreads), 0, s, a);
}

void launch_gather(const GatherArgs& a, hipStream_t s) {
    const dim3 grid((unsigned)gather_blocks_per_tile(a.g), a.ntiles);
    const bool per = a.g.periodic != 0;
    if (a.g.fdr == 2) {
        if (per) launch_gather_halo<3, true>(a, grid, s);
        else launch_gather_halo<3, false>(a, grid, s);
    } else {
        if (per) launch_gather_halo<2, true>(a, grid, s);
        else launch_gather_halo<2, false>(a, grid, s);
    }
}

}  // namespace cube
