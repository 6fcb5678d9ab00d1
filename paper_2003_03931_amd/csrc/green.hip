// Green's tables of the force split (Sec. II: F_G = F_s + F_l, F_s vanishing
// beyond the cut-off and F_l equal to F_G there; the split's form is left to
// the references, here the compact S2 split of Hockney & Eastwood).
//
//   S(xi)  = 12 (2 - 2 cos xi - xi sin xi) / xi^4, xi = k a_len / 2
//   coarse   G_c = -S^2 / k^2 (k != 0), 0 at k = 0            (FP64 table)
//   fine     K_f = IDFT_F[-(1 - S^2)/k^2] truncated to |d| <= a,
//            G_f = DFT_F[K_f]                                   (FP32 table)
//            (1 becomes S_pp^2 with the extended PP force of range pp_len:
//            the pair force then carries the part inside it, pp.hip)
// Both are real, even in every axis and symmetric under axis permutations, so
// one octant (n/2+1)^3 is stored; both already carry the 1/n^3 of the inverse
// transform.  Everything is built on the device in FP64.  The fine kernel
// uses separable cosine sums: K_f only needs |d| <= a, so no F^3 FP64 FFT.
#include <cmath>

#include "common.h"

namespace cube {

namespace {

__device__ double s2_window(double xi) {
    if (xi < 1.0) {
        // Taylor series: c_j = (-1)^j 12 (2j+2) / (2j+4)!
        const double c[10] = {1.0,
                              -1.0 / 15.0,
                              1.0 / 560.0,
                              -1.0 / 37800.0,
                              1.0 / 3991680.0,
                              -12.0 * 12.0 / 87178291200.0,
                              12.0 * 14.0 / 20922789888000.0,
                              -12.0 * 16.0 / 6402373705728000.0,
                              12.0 * 18.0 / 2432902008176640000.0,
                              -12.0 * 20.0 / 1.1240007277776077e21};
        const double x2 = xi * xi;
        double acc = 0.0;
        for (int j = 9; j >= 0; --j) acc = acc * x2 + c[j];
        return acc;
    }
    return 12.0 * (2.0 - 2.0 * cos(xi) - xi * sin(xi)) / (xi * xi * xi * xi);
}

// coarse octant: k = 2 pi m / L, divided by Nc^3
__global__ void k_coarse_green(int Nc, double L, double a_len, double* __restrict__ out) {
    const int M = Nc / 2 + 1;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (int64_t)M * M * M) return;
    const int mx = (int)(i % M), my = (int)((i / M) % M), mz = (int)(i / ((int64_t)M * M));
    const double dk = 2.0 * M_PI / L;
    const double k2 = dk * dk * (double)(mx * mx + my * my + mz * mz);
    double g = 0.0;
    if (k2 > 0.0) {
        const double S = s2_window(sqrt(k2) * a_len / 2.0);
        g = -S * S / k2;
    }
    out[i] = g / ((double)Nc * Nc * Nc);
}

// short-range continuum kernel on the fine octant, k = 2 pi m / (F h); with
// the extended PP force (pp_len > 0) the part inside pp_len is the pair
// force's: -(S_pp^2 - S^2) / k^2, k = 0 value -(a_len^2 - pp_len^2) / 30
__global__ void k_short_green(int F, double h, double a_len, double pp_len, double* __restrict__ out) {
    const int M = F / 2 + 1;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (int64_t)M * M * M) return;
    const int mx = (int)(i % M), my = (int)((i / M) % M), mz = (int)(i / ((int64_t)M * M));
    const double dk = 2.0 * M_PI / (F * h);
    const double k2 = dk * dk * (double)(mx * mx + my * my + mz * mz);
    double g;
    if (k2 > 0.0) {
        const double S = s2_window(sqrt(k2) * a_len / 2.0);
        double inner = 1.0;
        if (pp_len > 0.0) {
            const double Sp = s2_window(sqrt(k2) * pp_len / 2.0);
            inner = Sp * Sp;
        }
        g = -(inner - S * S) / k2;
    } else {
        g = -(a_len * a_len - pp_len * pp_len) / 30.0;
    }
    out[i] = g;
}

// One separable cosine sum along axis `ax` of a [d0][d1][d2] array (d2 fastest):
// out[..o..] = sum_{t < din} mult(t) cos(2 pi t o / F) in[..t..], o < dout.
// mult(t) = 1 for t == 0 (and t == F/2 when nyq), else 2 (folded even sums).
__global__ void k_cos_axis(const double* __restrict__ in, double* __restrict__ out, int d0, int d1, int d2, int ax,
                           int din, int dout, int F, int nyq) {
    int od[3] = {d0, d1, d2};
    od[ax] = dout;
    const int64_t total = (int64_t)od[0] * od[1] * od[2];
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= total) return;
    int o[3] = {(int)(i / ((int64_t)od[1] * od[2])), (int)((i / od[2]) % od[1]), (int)(i % od[2])};
    int id[3] = {d0, d1, d2};
    id[ax] = din;
    const int64_t s_in[3] = {(int64_t)id[1] * id[2], id[2], 1};
    int64_t base = 0;
    for (int k = 0; k < 3; ++k)
        if (k != ax) base += (int64_t)o[k] * s_in[k];
    double acc = 0.0;
    for (int t = 0; t < din; ++t) {
        const double mult = (t == 0 || (nyq && 2 * t == F)) ? 1.0 : 2.0;
        const int ph = (int)(((int64_t)t * o[ax]) % F);
        acc += mult * cospi(2.0 * (double)ph / (double)F) * in[base + (int64_t)t * s_in[ax]];
    }
    out[i] = acc;
}

__global__ void k_truncate_kernel(double* __restrict__ K, int A, int a, double scale) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (int64_t)A * A * A) return;
    const int dx = (int)(i / (A * A)), dy = (int)((i / A) % A), dz = (int)(i % A);
    K[i] = (dx * dx + dy * dy + dz * dz <= a * a) ? K[i] * scale : 0.0;
}

// FP32 copy of the octant, stored pencil-major [ky][kx][kz] (kz fastest):
// the z-pencil pass reads each pencil's kz profile as one contiguous run
__global__ void k_to_float_pencils(const double* __restrict__ in, float* __restrict__ out, int M, double scale) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (int64_t)M * M * M) return;
    const int fx = (int)(i % M), fy = (int)((i / M) % M), fz = (int)(i / ((int64_t)M * M));
    out[((int64_t)fy * M + fx) * M + fz] = (float)(in[i] * scale);
}

unsigned blocks_for(int64_t n) { return (unsigned)((n + 255) / 256); }

}  // namespace

void build_coarse_green(const Geom& g, double* octant, hipStream_t s) {
    const int M = g.Nc / 2 + 1;
    const double a_len = (double)g.a / g.f;
    hipLaunchKernelGGL(k_coarse_green, dim3(blocks_for((int64_t)M * M * M)), dim3(256), 0, s, g.Nc, (double)g.ns,
                       a_len, octant);
}

size_t fine_green_workspace_bytes(const Geom& g) {
    const int64_t M = g.F / 2 + 1;
    return (size_t)(2 * M * M * M) * sizeof(double) + 256;
}

void build_fine_green(const Geom& g, float* octant, void* ws, hipStream_t s) {
    const int F = g.F, M = F / 2 + 1, A = g.a + 1;
    const double h = 1.0 / g.f, a_len = (double)g.a / g.f;
    double* b0 = static_cast<double*>(ws);
    double* b1 = b0 + (int64_t)M * M * M;
    // G_s on the octant
    hipLaunchKernelGGL(k_short_green, dim3(blocks_for((int64_t)M * M * M)), dim3(256), 0, s, F, h, a_len,
                       (double)g.npp / g.f, b0);
    // K(d) = (1/F^3) sum_m G_s(m) cos(2 pi m.d / F), d in [0, a]^3
    hipLaunchKernelGGL(k_cos_axis, dim3(blocks_for((int64_t)A * M * M)), dim3(256), 0, s, b0, b1, M, M, M, 0, M, A,
                       F, 1);
    hipLaunchKernelGGL(k_cos_axis, dim3(blocks_for((int64_t)A * A * M)), dim3(256), 0, s, b1, b0, A, M, M, 1, M, A,
                       F, 1);
    hipLaunchKernelGGL(k_cos_axis, dim3(blocks_for((int64_t)A * A * A)), dim3(256), 0, s, b0, b1, A, A, M, 2, M, A,
                       F, 1);
    hipLaunchKernelGGL(k_truncate_kernel, dim3(blocks_for((int64_t)A * A * A)), dim3(256), 0, s, b1, A, g.a,
                       1.0 / ((double)F * F * F));
    // G_f(m) = sum_{|d| <= a} K(d) cos(2 pi m.d / F), m in [0, F/2]^3
    hipLaunchKernelGGL(k_cos_axis, dim3(blocks_for((int64_t)M * A * A)), dim3(256), 0, s, b1, b0, A, A, A, 0, A, M,
                       F, 0);
    hipLaunchKernelGGL(k_cos_axis, dim3(blocks_for((int64_t)M * M * A)), dim3(256), 0, s, b0, b1, M, A, A, 1, A, M,
                       F, 0);
    hipLaunchKernelGGL(k_cos_axis, dim3(blocks_for((int64_t)M * M * M)), dim3(256), 0, s, b1, b0, M, M, A, 2, A, M,
                       F, 0);
    // fold in the inverse-transform normalisation and round once to FP32
    hipLaunchKernelGGL(k_to_float_pencils, dim3(blocks_for((int64_t)M * M * M)), dim3(256), 0, s, b0, octant, M,
                       1.0 / ((double)F * F * F));
}

}  // namespace cube
