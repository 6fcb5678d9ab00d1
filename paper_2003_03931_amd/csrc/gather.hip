// Force interpolation, kick, drift and recount (Sec. II: the PM force is the
// long-range coarse-mesh part plus the short-range part of the particle's own
// tile; Sec. III-A: positions and velocities are re-encoded after the update).
//
// One workgroup per chunk (an x-row of coarse cells of one tile), whose
// particles are contiguous.  For each particle:
//   * decode (Eq. (2)) into fine-box and coarse coordinates, exactly;
//   * a = CIC-gather of -grad phi_f (tile box) + CIC-gather of -grad phi_c,
//     the gradients taken by 2-point central differences on the fly from the
//     potentials (no force mesh is stored);
//   * kick in FP64:  u' = clamp(rint((u s + a dt) / s'), -127, 127);
//   * drift in cell-local quanta, exactly in FP64:
//       X = m + 1/2 + ((u' s') (256/H)) dt,  q = floor(X),
//       carry = floor(q / 256), m' = q mod 256, cell' = cell + carry (periodic);
//   * write (m', u') at the same index of the second particle buffer, a move
//     code for the compaction and one count for the new cell.
#include "common.h"

namespace cube {

namespace {

struct FinePhi {
    const float* p;   // pair-packed complex mesh: value at 2*idx
    int F;
    bool wrap;
    __device__ float at(int x, int y, int z) const {
        if (wrap) { x = wrapi(x, F); y = wrapi(y, F); z = wrapi(z, F); }
        return p[2 * (((int64_t)z * F + y) * F + x)];
    }
};

struct CoarsePhi {
    const float* p;
    int N;
    __device__ float at(int x, int y, int z) const {
        x = wrapi(x, N); y = wrapi(y, N); z = wrapi(z, N);
        return p[2 * (((int64_t)z * N + y) * N + x)];
    }
};

// CIC gather of -grad(phi) with 2-point differences; i0/t per axis, inv2h = 1/(2 cell).
template <class Phi>
__device__ __forceinline__ void gather_force(const Phi& phi, const int i0[3], const float t[3], float inv2h,
                                             float out[3]) {
    const float w[3][2] = {{1.0f - t[0], t[0]}, {1.0f - t[1], t[1]}, {1.0f - t[2], t[2]}};
    float ax = 0.f, ay = 0.f, az = 0.f;
#pragma unroll
    for (int oz = 0; oz < 2; ++oz) {
#pragma unroll
        for (int oy = 0; oy < 2; ++oy) {
            const int y = i0[1] + oy, z = i0[2] + oz;
            const float xm = phi.at(i0[0] - 1, y, z), x0 = phi.at(i0[0], y, z);
            const float x1 = phi.at(i0[0] + 1, y, z), x2 = phi.at(i0[0] + 2, y, z);
            ax += w[1][oy] * w[2][oz] * (w[0][0] * (xm - x1) + w[0][1] * (x0 - x2));
        }
    }
#pragma unroll
    for (int oz = 0; oz < 2; ++oz) {
#pragma unroll
        for (int ox = 0; ox < 2; ++ox) {
            const int x = i0[0] + ox, z = i0[2] + oz;
            const float ym = phi.at(x, i0[1] - 1, z), y0 = phi.at(x, i0[1], z);
            const float y1 = phi.at(x, i0[1] + 1, z), y2 = phi.at(x, i0[1] + 2, z);
            ay += w[0][ox] * w[2][oz] * (w[1][0] * (ym - y1) + w[1][1] * (y0 - y2));
        }
    }
#pragma unroll
    for (int oy = 0; oy < 2; ++oy) {
#pragma unroll
        for (int ox = 0; ox < 2; ++ox) {
            const int x = i0[0] + ox, y = i0[1] + oy;
            const float zm = phi.at(x, y, i0[2] - 1), z0 = phi.at(x, y, i0[2]);
            const float z1 = phi.at(x, y, i0[2] + 1), z2 = phi.at(x, y, i0[2] + 2);
            az += w[0][ox] * w[1][oy] * (w[2][0] * (zm - z1) + w[2][1] * (z0 - z2));
        }
    }
    out[0] = ax * inv2h;
    out[1] = ay * inv2h;
    out[2] = az * inv2h;
}

template <class Phi>
__device__ __forceinline__ float gather_value(const Phi& phi, const int i0[3], const float t[3]) {
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

template <int MODE>
__global__ __launch_bounds__(256) void k_gather(GatherArgs A) {
    extern __shared__ int offs[];
    __shared__ double s_red[256 / kWave];
    const Geom& g = A.g;
    const int k = blockIdx.y;                        // tile within the batch
    const int tile = A.tile0 + k;
    const int64_t q = (int64_t)tile * g.Tc * g.Tc + blockIdx.x;
    const Chunk ch = chunk_of(g, q);
    for (int j = threadIdx.x; j <= g.Tc; j += blockDim.x) offs[j] = A.offsets[ch.c0 + j];
    __syncthreads();

    const FinePhi fphi{A.fine_pairs + (int64_t)(k >> 1) * 2 * (int64_t)g.F * g.F * g.F + (k & 1), g.F,
                       g.periodic != 0};
    const CoarsePhi cphi{reinterpret_cast<const float*>(A.coarse), g.Nc};
    const int D = 1 << g.log2D, halfD = D >> 1;
    const float invD = 1.0f / (float)D;
    const float inv2h = (float)g.f * 0.5f;                   // 1 / (2h)
    const float inv2H = (float)g.f / (2.0f * (float)g.r);    // 1 / (2H)

    double s = 0.0, s_next = 0.0;
    if (MODE == GATHER_STEP) { s = A.sc->s; s_next = A.sc->s_next; }
    const double q256H = 256.0 * g.f / g.r;                  // 256 / H
    const double dt = (double)A.dt;

    int umax = 0, sat = 0, cmax = 0, nfar = 0;
    double esum = 0.0;
    for (int p = offs[0] + threadIdx.x; p < offs[g.Tc]; p += blockDim.x) {
        const int j = find_cell(offs, g.Tc, p);
        const int cell[3] = {ch.cx0 + j, ch.cy, ch.cz};
        const int cbox[3] = {j + g.hc, ch.ly + g.hc, ch.lz + g.hc};   // tile-box coarse coords
        int m[3];
#pragma unroll
        for (int a = 0; a < 3; ++a) m[a] = A.in.m[a][p];
        int fi[3], ci[3];
        float ft[3], ct[3];
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            const int Pf = 2 * (cbox[a] * 256 + m[a]) + 1 - halfD;
            fi[a] = Pf >> g.log2D;
            ft[a] = (float)(Pf & (D - 1)) * invD;
            const int Pc = 2 * (cell[a] * 256 + m[a]) + 1 - 256;
            ci[a] = Pc >> 9;
            ct[a] = (float)(Pc & 511) * (1.0f / 512.0f);
        }
        if (MODE == GATHER_POTENTIAL) {
            esum += (double)gather_value(fphi, fi, ft) + (double)gather_value(cphi, ci, ct);
            continue;
        }
        float af[3], ac[3];
        gather_force(fphi, fi, ft, inv2h, af);
        gather_force(cphi, ci, ct, inv2H, ac);
        const float acc[3] = {af[0] + ac[0], af[1] + ac[1], af[2] + ac[2]};
        if (MODE == GATHER_FORCE) {
#pragma unroll
            for (int a = 0; a < 3; ++a) A.acc[3 * (int64_t)p + a] = acc[a];
            continue;
        }
        // kick (FP64) and requantise
        int un[3], carry[3], mn[3];
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            const double v = (double)A.in.u[a][p] * s + (double)acc[a] * dt;
            double w = rint(v / s_next);
            sat += fabs(w) > 127.0;
            w = fmin(fmax(w, -127.0), 127.0);
            un[a] = (int)w;
            umax = max(umax, abs(un[a]));
            // drift in cell-local quanta, exact in FP64
            const double X = ((double)m[a] + 0.5) + (((double)un[a] * s_next) * q256H) * dt;
            const int qq = (int)floor(X);
            carry[a] = qq >> 8;                  // floor division by 256
            mn[a] = qq & 255;
            cmax = max(cmax, abs(carry[a]));
        }
        int nc[3];
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            nc[a] = wrapi(cell[a] + carry[a], g.Nc);
            A.out.m[a][p] = (uint8_t)mn[a];
            A.out.u[a][p] = (int8_t)un[a];
        }
        if (A.out.ids) A.out.ids[p] = A.in.ids[p];
        const int64_t cn = canon(g, nc[0], nc[1], nc[2]);
        atomicAdd(&A.counts_new[cn], 1);
        const bool near = abs(carry[0]) <= 1 && abs(carry[1]) <= 1 && abs(carry[2]) <= 1;
        if (near) {
            A.dir[p] = (uint8_t)((carry[0] + 1) + 3 * (carry[1] + 1) + 9 * (carry[2] + 1));
        } else {
            A.dir[p] = 255;
            A.far_key[p] = (uint32_t)cn;
            ++nfar;
        }
    }

    if (MODE == GATHER_STEP) {
        umax = wave_max(umax);
        cmax = wave_max(cmax);
        sat = wave_sum(sat);
        nfar = wave_sum(nfar);
        if ((threadIdx.x & (kWave - 1)) == 0) {
            if (umax) atomicMax(&A.sc->max_u_next, umax);
            if (cmax) atomicMax(&A.sc->max_carry, cmax);
            if (sat) atomicAdd((unsigned long long*)&A.sc->saturations, (unsigned long long)sat);
            if (nfar) atomicAdd(&A.sc->far_count, nfar);
        }
    } else if (MODE == GATHER_POTENTIAL) {
        esum = wave_sum_d(esum);
        if ((threadIdx.x & (kWave - 1)) == 0) s_red[threadIdx.x / kWave] = esum;
        __syncthreads();
        if (threadIdx.x == 0) {
            double t = 0.0;
            for (int w = 0; w < (int)(blockDim.x / kWave); ++w) t += s_red[w];
            A.partial[(int64_t)k * gridDim.x + blockIdx.x] = t;
        }
    }
}

}  // namespace

void launch_gather(const GatherArgs& a, hipStream_t s) {
    const dim3 grid((unsigned)(a.g.Tc * a.g.Tc), a.ntiles);
    const size_t shm = (a.g.Tc + 1) * sizeof(int);
    if (a.mode == GATHER_STEP)
        hipLaunchKernelGGL(k_gather<GATHER_STEP>, grid, dim3(256), shm, s, a);
    else if (a.mode == GATHER_FORCE)
        hipLaunchKernelGGL(k_gather<GATHER_FORCE>, grid, dim3(256), shm, s, a);
    else
        hipLaunchKernelGGL(k_gather<GATHER_POTENTIAL>, grid, dim3(256), shm, s, a);
}

}  // namespace cube
