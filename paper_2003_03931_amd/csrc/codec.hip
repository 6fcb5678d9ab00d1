// Fixed-point particle codec (Sec. III-A, Eq. (2)).
//
// Positions: per axis the global quantum Q = floor(x * 256 / H) mod 256 N_c,
// stored as the byte m = Q mod 256 in canonical cell order; decoding gives the
// bin centre (Q + 1/2) H / 256, exact in FP32.  Velocities: one signed byte
// per axis, u = clamp(rint(v / s), -127, 127) with a power-of-two scale s, or
// (cell-mean codec) the FP32 velocities are placed in cell order here and
// encoded by vcodec.hip.
#include "common.h"

namespace cube {

namespace {

__global__ void k_encode_keys(Geom g, const float* __restrict__ pos, uint32_t* __restrict__ key,
                              uint32_t* __restrict__ qpack, uint32_t* __restrict__ idx, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double scale = 256.0 * g.f / g.r;          // 256 / H, a power of two
    const int64_t nq = 256 * (int64_t)g.Nc;
    int64_t q[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        double x = (double)pos[3 * i + k];
        int64_t v = (int64_t)floor(x * scale) % nq;
        q[k] = v < 0 ? v + nq : v;
    }
    key[i] = (uint32_t)canon(g, (int)(q[0] >> 8), (int)(q[1] >> 8), (int)(q[2] >> 8));
    qpack[i] = (uint32_t)(q[0] & 255) | ((uint32_t)(q[1] & 255) << 8) | ((uint32_t)(q[2] & 255) << 16);
    idx[i] = (uint32_t)i;
}

__global__ void k_absmax(const float* __restrict__ v, int64_t n, uint32_t* __restrict__ out) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    uint32_t m = 0;
    for (; i < n; i += stride) m = max(m, __float_as_uint(fabsf(v[i])));
    int mi = wave_max((int)m);   // non-negative floats order like their bits
    if ((threadIdx.x & (kWave - 1)) == 0) atomicMax(out, (uint32_t)mi);
}

__global__ void k_count_keys(const uint32_t* __restrict__ key, int64_t n, int32_t* __restrict__ counts) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) atomicAdd(&counts[key[i]], 1);
}

__global__ void k_scatter_compressed(Geom g, const uint32_t* __restrict__ perm,
                                     const uint32_t* __restrict__ qpack, const float* __restrict__ vel,
                                     double s_v, Planes out, StepScalars* sc, int64_t n) {
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int sat = 0, umax = 0;
    if (j < n) {
        const uint32_t src = min(perm[j], (uint32_t)(n - 1));
        const uint32_t qp = qpack[src];
        out.m[0][j] = (uint8_t)(qp & 255);
        out.m[1][j] = (uint8_t)((qp >> 8) & 255);
        out.m[2][j] = (uint8_t)((qp >> 16) & 255);
        if (out.v[0]) {
#pragma unroll
            for (int k = 0; k < 3; ++k) out.v[k][j] = vel[3 * (int64_t)src + k];
        } else {
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                double w = rint((double)vel[3 * (int64_t)src + k] / s_v);
                sat += fabs(w) > 127.0;
                w = fmin(fmax(w, -127.0), 127.0);
                int u = (int)w;
                umax = max(umax, abs(u));
                out.u[k][j] = (int8_t)u;
            }
        }
        if (out.ids) out.ids[j] = src;
    }
    if (out.v[0]) return;                    // codes are written by the cell-mean encoder
    sat = wave_sum(sat);
    umax = wave_max(umax);
    if ((threadIdx.x & (kWave - 1)) == 0) {
        if (sat) atomicAdd((unsigned long long*)&sc->saturations, (unsigned long long)sat);
        // one address for the whole grid: skip the atomic when the (monotone)
        // maximum already covers this wave
        if (umax > *(volatile int32_t*)&sc->max_u) atomicMax(&sc->max_u, umax);
    }
}

// One block per chunk (x-row of cells in a tile).
__global__ __launch_bounds__(256) void k_decode(Geom g, const int32_t* __restrict__ offsets, Planes in,
                                                const StepScalars* __restrict__ sc, VelCells vcell,
                                                float* __restrict__ pos, float* __restrict__ vel) {
    extern __shared__ int offs[];
    const Chunk ch = chunk_of(g, blockIdx.x);
    for (int j = threadIdx.x; j <= g.Tc; j += blockDim.x) offs[j] = offsets[ch.c0 + j];
    __syncthreads();
    const float H256 = (float)g.r / (float)(256 * g.f);   // H / 256, a power of two
    const float s = (float)sc->s;
    for (int p = offs[0] + threadIdx.x; p < offs[g.Tc]; p += blockDim.x) {
        const int j = find_cell(offs, g.Tc, p);
        const int c[3] = {ch.cx0 + j, ch.cy, ch.cz};
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            const int q = c[k] * 256 + in.m[k][p];
            pos[3 * (int64_t)p + k] = ((float)q + 0.5f) * H256;
            vel[3 * (int64_t)p + k] = g.vcodec
                                          ? (float)vc_decode(vcell.vc[k][ch.c0 + j], sc->s, vcell.tab, in.u[k][p])
                                          : (float)in.u[k][p] * s;
        }
    }
}

}  // namespace

void launch_encode_keys(const Geom& g, const float* pos, uint32_t* key, uint32_t* qpack, uint32_t* idx,
                        int64_t n, hipStream_t s) {
    hipLaunchKernelGGL(k_encode_keys, dim3(grid1d(n, 256)), dim3(256), 0, s, g, pos, key, qpack, idx, n);
}

void launch_absmax_f32(const float* v, int64_t n, uint32_t* out_bits, hipStream_t s) {
    unsigned blocks = grid1d(n, 256);
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(k_absmax, dim3(blocks), dim3(256), 0, s, v, n, out_bits);
}

void launch_count_keys(const uint32_t* key, int64_t n, int32_t* counts, hipStream_t s) {
    hipLaunchKernelGGL(k_count_keys, dim3(grid1d(n, 256)), dim3(256), 0, s, key, n, counts);
}

void launch_scatter_compressed(const Geom& g, const uint32_t* perm, const uint32_t* qpack, const float* vel,
                               double s_v, Planes out, int32_t* /*counts*/, StepScalars* sc, int64_t n,
                               hipStream_t st) {
    hipLaunchKernelGGL(k_scatter_compressed, dim3(grid1d(n, 256)), dim3(256), 0, st, g, perm, qpack, vel,
                       s_v, out, sc, n);
}

void launch_decode(const Geom& g, const int32_t* offsets, Planes in, const StepScalars* sc,
                   const VelCells& vcell, float* pos, float* vel, hipStream_t s) {
    const int64_t chunks = g.ncells / g.Tc;
    hipLaunchKernelGGL(k_decode, dim3((unsigned)chunks), dim3(256), (g.Tc + 1) * sizeof(int), s, g, offsets,
                       in, sc, vcell, pos, vel);
}

}  // namespace cube
