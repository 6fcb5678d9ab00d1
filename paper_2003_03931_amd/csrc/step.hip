// Per-step scalar bookkeeping and FP64 diagnostics.
//
// Velocity scale update before each kick: s' = pow2ceil(h_v M s / 127) with M
// the max |u| left by the previous kick (kept at s when M = 0); evaluated in
// FP64 on the device so a multi-step call never waits for the host.
// Diagnostics: momentum and kinetic energy of the decoded velocities summed in
// FP64 in a fixed order (per-chunk partials, then one ordered reduction);
// power-spectrum shells binned in FP64.
#include <cmath>

#include "common.h"

namespace cube {

namespace {

__device__ double pow2ceil_d(double x) {
    int e;
    const double m = frexp(x, &e);      // x = m 2^e, m in [0.5, 1)
    return m == 0.5 ? ldexp(1.0, e - 1) : ldexp(1.0, e);
}

__device__ __forceinline__ bool halted(const StepScalars* sc) { return *(volatile const int32_t*)&sc->halt != 0; }

__global__ void k_prologue(StepScalars* sc, float hv) {
    if (threadIdx.x != 0 || halted(sc)) return;
    const int M = sc->max_u;
    const double s = sc->s;
    sc->s_next = (M == 0) ? s : pow2ceil_d(((double)hv * (double)M) * s / 127.0);
    sc->max_u_next = 0;
    sc->far_count = 0;
    sc->max_carry = 0;
    sc->overflow = 0;
    sc->sat_step = 0;
    for (int i = 0; i < 64; ++i) {
        sc->umax_slot[i] = 0;
        sc->cmax_slot[i] = 0;
    }
}

__global__ void k_decide(StepScalars* sc, int32_t fast_max_count) {
    if (threadIdx.x != 0 || halted(sc)) return;
    if (sc->overflow) sc->halt = 2;
    else if (sc->far_count > 0 || sc->max_count > fast_max_count || sc->new_max_count > fast_max_count) sc->halt = 1;
}

// counts <- counts_new and offsets <- offsets_new, 16 bytes at a time where aligned
__global__ __launch_bounds__(256) void k_commit_cells(const int32_t* __restrict__ cn, const int32_t* __restrict__ on,
                                                      int32_t* __restrict__ c, int32_t* __restrict__ o, int64_t ncells,
                                                      const StepScalars* sc) {
    if (halted(sc)) return;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const int64_t n4 = ncells / 4;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n4; i += stride) {
        reinterpret_cast<int4*>(c)[i] = reinterpret_cast<const int4*>(cn)[i];
        reinterpret_cast<int4*>(o)[i] = reinterpret_cast<const int4*>(on)[i];
    }
    for (int64_t i = 4 * n4 + (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i <= ncells; i += stride) {
        if (i < ncells) c[i] = cn[i];
        o[i] = on[i];
    }
}

__global__ void k_epilogue(StepScalars* sc, int vcodec, int planned_wide, int planned_f16, double wide_cut,
                           double f16_cut, double f3) {
    if (threadIdx.x != 0 || halted(sc)) return;
    int um = sc->max_u_next, cm = sc->max_carry;
    for (int i = 0; i < 64; ++i) {
        um = max(um, sc->umax_slot[i]);
        cm = max(cm, sc->cmax_slot[i]);
    }
    if (!vcodec) {
        sc->s = sc->s_next;
        sc->max_u = um;
    }
    sc->max_carry = cm;
    sc->saturations += sc->sat_step;
    sc->sat_step = 0;
    sc->max_count = sc->new_max_count;
    sc->max_block8 = sc->new_max_block8;
    sc->steps_done += 1;
    // the next step was enqueued for narrower accumulators or FP16 densities
    const double b8 = (double)sc->max_block8;
    if ((!planned_wide && b8 >= wide_cut) || (planned_f16 && f3 * b8 + 1.0 >= f16_cut)) sc->halt = 3;
}

__global__ void k_strided_copy(const int32_t* __restrict__ in, int64_t stride, int32_t* __restrict__ out, int64_t n,
                               const int32_t* gate) {
    if (gate && *(volatile const int32_t*)gate) return;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        out[i] = in[i * stride];
}

__global__ void k_fill(int32_t* p, int32_t v, int64_t n, const int32_t* gate) {
    if (gate && *(volatile const int32_t*)gate) return;
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (; i < n; i += stride) p[i] = v;
}

// per chunk: sum v_x, v_y, v_z, v^2 in FP64 (v = u s, or the cell-mean
// decode v_c + sigma tan(u pi / 255))
__global__ __launch_bounds__(256) void k_moments(Geom g, const int32_t* __restrict__ offsets, Planes p,
                                                 const StepScalars* __restrict__ sc, VelCells vcell,
                                                 double* __restrict__ partial) {
    extern __shared__ int offs[];
    __shared__ double red[4][256 / kWave];
    const int64_t c0 = (int64_t)blockIdx.x * g.Tc;
    for (int j = threadIdx.x; j <= g.Tc; j += blockDim.x) offs[j] = offsets[c0 + j];
    __syncthreads();
    const int lo = offs[0], hi = offs[g.Tc];
    const double s = sc->s;
    double a[4] = {0.0, 0.0, 0.0, 0.0};
    for (int i = lo + threadIdx.x; i < hi; i += blockDim.x) {
        const int64_t c = g.vcodec ? c0 + find_cell(offs, g.Tc, i) : 0;
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            const double v = g.vcodec ? vc_decode(vcell.vc[k][c], s, vcell.tab, p.u[k][i]) : (double)p.u[k][i] * s;
            a[k] += v;
            a[3] += v * v;
        }
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const double v = wave_sum_d(a[k]);
        if ((threadIdx.x & (kWave - 1)) == 0) red[k][threadIdx.x / kWave] = v;
    }
    __syncthreads();
    if (threadIdx.x < 4) {
        double t = 0.0;
        for (int w = 0; w < (int)(blockDim.x / kWave); ++w) t += red[threadIdx.x][w];
        partial[(int64_t)blockIdx.x * 4 + threadIdx.x] = t;
    }
}

// out[c] = sum_b partial[b * width + c], fixed order
__global__ __launch_bounds__(256) void k_reduce_partials(const double* __restrict__ partial, int nblocks, int width,
                                                         double* __restrict__ out) {
    __shared__ double red[256 / kWave];
    const int c = blockIdx.x;
    double acc = 0.0;
    for (int b = threadIdx.x; b < nblocks; b += blockDim.x) acc += partial[(int64_t)b * width + c];
    acc = wave_sum_d(acc);
    if ((threadIdx.x & (kWave - 1)) == 0) red[threadIdx.x / kWave] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int w = 0; w < (int)(blockDim.x / kWave); ++w) t += red[w];
        out[c] = t;
    }
}

// floor(sqrt(v)) of a non-negative integer, exactly
__device__ __forceinline__ long isqrt_floor(long v) {
    long q = (long)sqrt((double)v);
    while (q * q > v) --q;
    while ((q + 1) * (q + 1) <= v) ++q;
    return q;
}

// One block per z-plane: shell sums of |dk|^2 / n^3, mode counts and |k|
// sums.  A mode with integer |m|^2 = r2 falls in shell j = floor(sqrt(r2) +
// 1/2) exactly when j^2 - j + 1 <= r2 <= j^2 + j, so each thread owns whole
// shells and walks a shell's modes of the plane in a fixed order (rows m_y
// ascending, then |m_x| ascending, + before -): the sums do not depend on
// scheduling, and the spectrum is reproducible bit for bit.
__global__ __launch_bounds__(256) void k_power_bins(const float2* __restrict__ dk, int n, int nbins,
                                                    double* __restrict__ partial) {
    const int z = blockIdx.x;
    const long mz = z <= n / 2 - 1 ? z : z - n;
    const int half = n / 2;
    const double inv_n3 = 1.0 / ((double)n * n * n);
    const double kf = 2.0 * M_PI / n;
    for (int j = (int)threadIdx.x + 1; j <= nbins; j += blockDim.x) {
        double ps = 0.0, ks = 0.0, cs = 0.0;
        const long A0 = (long)j * j - j + 1 - mz * mz, B0 = (long)j * j + j - mz * mz;
        if (B0 >= 0) {
            const long ymax = isqrt_floor(B0);
            for (long my = -ymax; my <= ymax; ++my) {
                if (my < -half || my > half - 1) continue;
                const long A = A0 - my * my, B = B0 - my * my;
                if (B < 0) continue;
                long lo = 0;
                if (A > 0) {
                    lo = isqrt_floor(A - 1) + 1;                        // ceil(sqrt(A))
                }
                const long hi = isqrt_floor(B);
                const int y = (int)(my >= 0 ? my : my + n);
                for (long mx = lo; mx <= hi; ++mx) {
                    const double r = sqrt((double)(mx * mx + my * my + mz * mz));
#pragma unroll
                    for (int sgn = 0; sgn < 2; ++sgn) {
                        if (sgn == 1 && mx == 0) break;
                        const long sx = sgn ? -mx : mx;
                        if (sx < -half || sx > half - 1) continue;
                        const int x = (int)(sx >= 0 ? sx : sx + n);
                        const float2 v = dk[((int64_t)z * n + y) * n + x];
                        ps += ((double)v.x * v.x + (double)v.y * v.y) * inv_n3;
                        ks += r * kf;
                        cs += 1.0;
                    }
                }
            }
        }
        partial[(int64_t)z * 3 * nbins + (j - 1)] = ps;
        partial[(int64_t)z * 3 * nbins + nbins + (j - 1)] = ks;
        partial[(int64_t)z * 3 * nbins + 2 * nbins + (j - 1)] = cs;
    }
}

}  // namespace

void launch_step_prologue(StepScalars* sc, float v_headroom, hipStream_t s) {
    hipLaunchKernelGGL(k_prologue, dim3(1), dim3(64), 0, s, sc, v_headroom);
}

void launch_step_decide(StepScalars* sc, int32_t fast_max_count, hipStream_t s) {
    hipLaunchKernelGGL(k_decide, dim3(1), dim3(64), 0, s, sc, fast_max_count);
}

void launch_commit_cells(const int32_t* counts_new, const int32_t* offsets_new, int32_t* counts, int32_t* offsets,
                         int64_t ncells, const StepScalars* sc, hipStream_t s) {
    unsigned blocks = grid1d(ncells / 4 + 1, 256);
    if (blocks > 8192) blocks = 8192;
    hipLaunchKernelGGL(k_commit_cells, dim3(blocks), dim3(256), 0, s, counts_new, offsets_new, counts, offsets, ncells,
                       sc);
}

void launch_step_epilogue(StepScalars* sc, const Geom& g, int vcodec, bool planned_wide, bool planned_f16,
                          hipStream_t s) {
    // 32-bit fine accumulators hold D^3 units per particle of a 2x2x2 block of
    // coarse cells; FP16 density spectra hold f^3 per particle of such a block
    const double wide_cut = std::ldexp(1.0, 32 - 3 * g.log2D);
    const double f3 = (double)g.f * g.f * g.f;
    hipLaunchKernelGGL(k_epilogue, dim3(1), dim3(64), 0, s, sc, vcodec, planned_wide ? 1 : 0, planned_f16 ? 1 : 0,
                       wide_cut, 32768.0, f3);
}

void launch_strided_copy(const int32_t* in, int64_t stride, int32_t* out, int64_t n, hipStream_t s,
                         const int32_t* gate) {
    unsigned blocks = grid1d(n, 256);
    if (blocks > 1024) blocks = 1024;
    hipLaunchKernelGGL(k_strided_copy, dim3(blocks), dim3(256), 0, s, in, stride, out, n, gate);
}

void launch_fill_i32(int32_t* p, int32_t v, int64_t n, hipStream_t s, const int32_t* gate) {
    unsigned blocks = grid1d(n, 256);
    if (blocks > 65536) blocks = 65536;
    hipLaunchKernelGGL(k_fill, dim3(blocks), dim3(256), 0, s, p, v, n, gate);
}

void launch_moments(const Geom& g, const int32_t* offsets, Planes p, const StepScalars* sc,
                    const VelCells& vcell, double* partial, int nblocks, hipStream_t s) {
    hipLaunchKernelGGL(k_moments, dim3(nblocks), dim3(256), (g.Tc + 1) * sizeof(int), s, g, offsets, p, sc, vcell,
                       partial);
}

void launch_reduce_partials(const double* partial, int nblocks, int width, double* out, hipStream_t s) {
    hipLaunchKernelGGL(k_reduce_partials, dim3(width), dim3(256), 0, s, partial, nblocks, width, out);
}

void launch_power_bins(const float2* dk, int n, int nbins, double* partial, int /*nparts*/, hipStream_t s) {
    hipLaunchKernelGGL(k_power_bins, dim3(n), dim3(256), 0, s, dk, n, nbins, partial);
}

}  // namespace cube
