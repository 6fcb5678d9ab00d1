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
//   3. u = clamp(rint(atan~((v - v_c) / sigma) * (255 / pi)), -127, 127), atan~
//      the quadratic arctangent of Eq. (4) reflected outside [-1, 1]; a
//      component beyond the last code's value sigma tan(127 pi / 255) is
//      counted as saturated.
// Eq. (4)'s error (<= 0.0038 rad) is below half a code's angle, so every code
// re-encodes to itself.  One workgroup per 256 consecutive canonical cells:
// the mean pass stages the cells' velocities in LDS with coalesced loads and
// gives each cell to one thread, which sums its particles in order; sigma is
// a fixed-order reduction of the per-workgroup sums; the encode pass gives
// each particle to one thread.
#include <cmath>

#include "common.h"

namespace cube {

namespace {

constexpr double kAngle = M_PI / 255.0;
constexpr double kCodesPerRadian = 255.0 / M_PI;
constexpr int kCells = 256;              // cells (and threads) per workgroup
constexpr int kStage = 2048;             // particles whose velocities are staged in LDS
constexpr int kSigmaThreads = 1024;

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

// offsets of the workgroup's cells [c0, c0 + nc] into s_off
__device__ __forceinline__ int stage_offsets(const Geom& g, const int32_t* offsets, int* s_off, int64_t& c0) {
    c0 = (int64_t)blockIdx.x * kCells;
    const int nc = (int)min<int64_t>(kCells, g.ncells - c0);
    for (int j = threadIdx.x; j <= nc; j += blockDim.x) s_off[j] = offsets[c0 + j];
    return nc;
}

// cell means into vc; sum of squared deviations of the workgroup into partial
__global__ __launch_bounds__(kCells) void k_vc_mean(Geom g, const int32_t* __restrict__ offsets, Planes p,
                                                    VelCells vcell, double* __restrict__ partial, const int32_t* gate) {
    if (gate && *(volatile const int32_t*)gate) return;
    __shared__ int s_off[kCells + 1];
    __shared__ float s_v[3][kStage];
    __shared__ double red[kCells / kWave];
    int64_t c0;
    const int nc = stage_offsets(g, offsets, s_off, c0);
    __syncthreads();
    const int lo = s_off[0], tot = s_off[nc] - lo;
    const bool staged = tot <= kStage;
    if (staged)
        for (int e = threadIdx.x; e < tot; e += kCells)
#pragma unroll
            for (int k = 0; k < 3; ++k) s_v[k][e] = p.v[k][lo + e];
    __syncthreads();
    double acc = 0.0;
    if ((int)threadIdx.x < nc) {
        const int64_t c = c0 + threadIdx.x;
        const int a = s_off[threadIdx.x] - lo, b = s_off[threadIdx.x + 1] - lo;
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            const float* v = staged ? s_v[k] : p.v[k] + lo;
            double sum = 0.0;
            for (int q = a; q < b; ++q) sum += (double)v[q];
            const float mean = b > a ? (float)(sum / (double)(b - a)) : 0.0f;
            vcell.vc[k][c] = mean;
            for (int q = a; q < b; ++q) {
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
        for (int w = 0; w < kCells / kWave; ++w) t += red[w];
        partial[blockIdx.x] = t;
    }
}

// sigma from the per-workgroup sums (fixed order); max |u| restarts for the encode
__global__ __launch_bounds__(kSigmaThreads) void k_vc_sigma(const double* __restrict__ partial, int nparts,
                                                            int64_t ncomp, StepScalars* sc, const int32_t* gate) {
    if (gate && *(volatile const int32_t*)gate) return;
    __shared__ double red[kSigmaThreads / kWave];
    double acc = 0.0;
    for (int b = threadIdx.x; b < nparts; b += kSigmaThreads) acc += partial[b];
    acc = wave_sum_d(acc);
    if ((threadIdx.x & (kWave - 1)) == 0) red[threadIdx.x / kWave] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int w = 0; w < kSigmaThreads / kWave; ++w) t += red[w];
        const double rms = ncomp > 0 ? sqrt(t / (double)ncomp) : 0.0;
        const double sigma = rms > 0.0 ? pow2ceil_vc(rms) : 1.0;
        sc->s = sigma;
        sc->s_next = sigma;
        sc->max_u = 0;
    }
}

__global__ __launch_bounds__(kCells) void k_vc_encode(Geom g, const int32_t* __restrict__ offsets, Planes p,
                                                      VelCells vcell, StepScalars* sc, const int32_t* gate) {
    if (gate && *(volatile const int32_t*)gate) return;
    __shared__ int s_off[kCells + 1];
    int64_t c0;
    const int nc = stage_offsets(g, offsets, s_off, c0);
    __syncthreads();
    const double sigma = sc->s, inv_sigma = 1.0 / sigma;     // exact: sigma is a power of two
    const double dmax = sigma * vcell.tab[254];              // last code's value
    int sat = 0, umax = 0;
    for (int q = s_off[0] + threadIdx.x; q < s_off[nc]; q += kCells) {
        const int64_t c = c0 + find_cell_fixed<8>(s_off, nc, q);
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            const double d = (double)p.v[k][q] - (double)vcell.vc[k][c];
            sat += fabs(d) > dmax;
            double w = rint(fast_atan_d(d * inv_sigma) * kCodesPerRadian);
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
        // the maximum only grows: skip the atomic (one address for the whole
        // grid) when the value already there is at least this wave's
        if (umax > *(volatile int32_t*)&sc->max_u) atomicMax(&sc->max_u, umax);
    }
}

}  // namespace

void vc_table_host(double* tab) {
    for (int u = -127; u <= 127; ++u) tab[u + 127] = std::tan((double)u * kAngle);
}

int vc_partials(const Geom& g) { return (int)((g.ncells + kCells - 1) / kCells); }

void launch_vc_encode(const Geom& g, const int32_t* offsets, Planes p, const VelCells& vcell, StepScalars* sc,
                      double* partial, hipStream_t s, bool gated) {
    const int32_t* gate = gated ? &sc->halt : nullptr;
    const int blocks = vc_partials(g);
    hipLaunchKernelGGL(k_vc_mean, dim3((unsigned)blocks), dim3(kCells), 0, s, g, offsets, p, vcell, partial, gate);
    hipLaunchKernelGGL(k_vc_sigma, dim3(1), dim3(kSigmaThreads), 0, s, partial, blocks, 3 * g.n, sc, gate);
    hipLaunchKernelGGL(k_vc_encode, dim3((unsigned)blocks), dim3(kCells), 0, s, g, offsets, p, vcell, sc, gate);
}

}  // namespace cube
