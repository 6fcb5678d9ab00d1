// Cell-mean velocity codec (Sec. III-A, Eq. (3)) with the fast arctangent of
// Eq. (4).
//
// A cell-ordered state carries, per coarse cell, the FP32 mean velocity v_c
// of its particles and, per particle and axis, one signed byte u with
//     v = v_c + sigma tan(u pi / 255),    u in [-127, 127],
// sigma a power of two per box.  Encoding from FP32 velocities v:
//   1. v_c: FP64 sum of the cell's velocities in storage order, divided by the
//      count, rounded to FP32 (0 for an empty cell);
//   2. sigma: smallest power of two >= the rms of all components of
//      v - v_c (1 when they are all zero);
//   3. u = clamp(rint(atan~((v - v_c) / sigma) 255 / pi), -127, 127), atan~
//      the quadratic arctangent of Eq. (4) reflected outside [-1, 1]; a
//      component beyond the last code's value sigma tan(127 pi / 255) is
//      counted as saturated.
// Eq. (4)'s error (<= 0.0038 rad) is below half a code's angle, so every code
// re-encodes to itself.  One workgroup per chunk of Tc cells (a tile row);
// the mean pass gives each cell to one thread, which sums its particles in
// order.
#include <cmath>

#include "common.h"

namespace cube {

namespace {

constexpr double kAngle = M_PI / 255.0;
constexpr int kMeanThreads = 64;
constexpr int kEncThreads = 256;

__device__ double pow2ceil_vc(double x) {
    int e;
    const double m = frexp(x, &e);
    return m == 0.5 ? ldexp(1.0, e - 1) : ldexp(1.0, e);
}

// Eq. (4), one rounding per operation in the order written (no contraction)
__device__ double fast_atan_d(double x) {
#pragma clang fp contract(off)
    const double ax = fabs(x);
    if (ax <= 1.0) return (M_PI / 4.0) * x + 0.273 * x * (1.0 - ax);
    const double r = 1.0 / x;
    const double half_pi = x > 0.0 ? M_PI / 2.0 : -(M_PI / 2.0);
    return half_pi - (M_PI / 4.0) * r - 0.273 * r * (1.0 - fabs(r));
}

// per chunk of Tc cells: cell means into vc, sum of squared deviations into
// partial[chunk]
__global__ __launch_bounds__(kMeanThreads) void k_vc_mean(Geom g, const int32_t* __restrict__ offsets, Planes p,
                                                          VelCells vcell, double* __restrict__ partial) {
    __shared__ double red[kMeanThreads / kWave];
    const int64_t c0 = (int64_t)blockIdx.x * g.Tc;
    double acc = 0.0;
    for (int j = threadIdx.x; j < g.Tc; j += kMeanThreads) {
        const int64_t c = c0 + j;
        const int lo = offsets[c], hi = offsets[c + 1], n = hi - lo;
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            const float* v = p.v[k];
            double sum = 0.0;
            for (int q = lo; q < hi; ++q) sum += (double)v[q];
            const float mean = n > 0 ? (float)(sum / (double)n) : 0.0f;
            vcell.vc[k][c] = mean;
            for (int q = lo; q < hi; ++q) {
                const double d = (double)v[q] - (double)mean;
                acc += d * d;
            }
        }
    }
    acc = wave_sum_d(acc);
    if ((threadIdx.x & (kWave - 1)) == 0) red[threadIdx.x / kWave] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int w = 0; w < kMeanThreads / kWave; ++w) t += red[w];
        partial[blockIdx.x] = t;
    }
}

// sigma from the per-chunk sums (fixed order); max |u| restarts for the encode
__global__ __launch_bounds__(256) void k_vc_sigma(const double* __restrict__ partial, int nchunks, int64_t ncomp,
                                                  StepScalars* sc) {
    __shared__ double red[256 / kWave];
    double acc = 0.0;
    for (int b = threadIdx.x; b < nchunks; b += blockDim.x) acc += partial[b];
    acc = wave_sum_d(acc);
    if ((threadIdx.x & (kWave - 1)) == 0) red[threadIdx.x / kWave] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int w = 0; w < (int)(blockDim.x / kWave); ++w) t += red[w];
        const double rms = ncomp > 0 ? sqrt(t / (double)ncomp) : 0.0;
        const double sigma = rms > 0.0 ? pow2ceil_vc(rms) : 1.0;
        sc->s = sigma;
        sc->s_next = sigma;
        sc->max_u = 0;
    }
}

__global__ __launch_bounds__(kEncThreads) void k_vc_encode(Geom g, const int32_t* __restrict__ offsets, Planes p,
                                                           VelCells vcell, StepScalars* sc) {
    extern __shared__ int offs[];
    const int64_t c0 = (int64_t)blockIdx.x * g.Tc;
    for (int j = threadIdx.x; j <= g.Tc; j += blockDim.x) offs[j] = offsets[c0 + j];
    __syncthreads();
    const double sigma = sc->s;
    const double dmax = sigma * vcell.tab[254];          // last code's value
    int sat = 0, umax = 0;
    for (int q = offs[0] + threadIdx.x; q < offs[g.Tc]; q += blockDim.x) {
        const int64_t c = c0 + find_cell(offs, g.Tc, q);
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            const double d = (double)p.v[k][q] - (double)vcell.vc[k][c];
            sat += fabs(d) > dmax;
            double w = rint(fast_atan_d(d / sigma) / kAngle);
            w = fmin(fmax(w, -127.0), 127.0);
            const int u = (int)w;
            umax = max(umax, abs(u));
            p.u[k][q] = (int8_t)u;
        }
    }
    sat = wave_sum(sat);
    umax = wave_max(umax);
    if ((threadIdx.x & (kWave - 1)) == 0) {
        if (sat) atomicAdd((unsigned long long*)&sc->saturations, (unsigned long long)sat);
        if (umax) atomicMax(&sc->max_u, umax);
    }
}

}  // namespace

void vc_table_host(double* tab) {
    for (int u = -127; u <= 127; ++u) tab[u + 127] = std::tan((double)u * kAngle);
}

void launch_vc_encode(const Geom& g, const int32_t* offsets, Planes p, const VelCells& vcell, StepScalars* sc,
                      double* partial, hipStream_t s) {
    const int chunks = (int)(g.ncells / g.Tc);
    hipLaunchKernelGGL(k_vc_mean, dim3((unsigned)chunks), dim3(kMeanThreads), 0, s, g, offsets, p, vcell, partial);
    hipLaunchKernelGGL(k_vc_sigma, dim3(1), dim3(256), 0, s, partial, chunks, 3 * g.n, sc);
    hipLaunchKernelGGL(k_vc_encode, dim3((unsigned)chunks), dim3(kEncThreads), (g.Tc + 1) * sizeof(int), s, g,
                       offsets, p, vcell, sc);
}

}  // namespace cube
