// Extended PP force (Sec. II, optional PP module; Sec. III-B, pair distances
// from the compressed integer positions).
//
// Every pair of particles closer than r_pp = n_pp fine cells attracts by
//     F_pp(r) = F_G(r) - F_l(r; r_pp),
// F_l(r; D) the attraction of two S2 clouds of diameter D (Hockney &
// Eastwood's reference force), which equals F_G from r = D on; the fine
// mesh's kernel leaves this part out (green.hip).  With xi = 2 r / D:
//     4 pi D^2 F_l = (224 xi - 224 xi^3 + 70 xi^4 + 48 xi^5 - 21 xi^6) / 35,  xi <= 1
//                  = (12/xi^2 - 224 + 896 xi - 840 xi^2 + 224 xi^3 + 70 xi^4
//                     - 48 xi^5 + 7 xi^6) / 35,                            1 <= xi <= 2.
// r_pp <= H, so a particle's partners lie in its own or the adjacent coarse
// cells.  Positions stay in the fixed-point format: per axis the separation
// is 256 (cell' - cell) + m' - m quanta (|.| < 512), the squared distance is
// an exact integer from a packed 16-bit dot product (the CDNA analogue of
// the paper's 8-bit VNNI distances), and only pairs inside r_pp reach the
// FP32 force polynomial.  Coincident particles (and a particle with itself)
// exert nothing.
//
// One workgroup per x-row of Tc coarse cells of a tile (a contiguous run of
// the canonical order).  It first stages the packed positions of the 3 x 3
// neighbouring rows, Tc + 2 cells each, in LDS (one coalesced pass; a row's
// middle Tc cells are one particle range); per axis a thread then visits its
// own cell and the neighbour on the side its r_pp sphere reaches, reading the
// partners from LDS.  A workgroup whose neighbourhood holds more than kPPCap
// particles reads them from global memory instead.  The accelerations go to
// three FP32 planes in canonical order, which the gather adds to the mesh
// force before the kick.
#include <cmath>

#include "common.h"

namespace cube {

namespace {

typedef short v2i16 __attribute__((ext_vector_type(2)));

constexpr int kPPThreads = 256;
constexpr int kPPCap = 4096;     // neighbour particles a workgroup stages in LDS

struct PPParams {
    int reach;        // r_pp in position quanta: 256 n_pp / r
    int reach2;       // its square
    float two_over;   // 2 / reach: xi per quantum
    float amp;        // (256 / H)^2 / (4 pi) / 140: quanta to spacings, 4 pi G = 1
};

// F_pp / r per quantum of separation, in units of amp, for 0 < u < reach:
// F_pp = F_G R(xi) / 140 with R = 140 - 35 xi^2 (4 pi D^2 F_l), i.e.
//     R = 140 - xi^3 (224 - 224 xi^2 + 70 xi^3 + 48 xi^4 - 21 xi^5)   (xi <= 1)
//     R = t^5 (168 - 182 t + 64 t^2 - 7 t^3),  t = 2 - xi           (1 <= xi < 2)
// The second line is the outer branch rewritten about xi = 2, where the pair
// force vanishes to fifth order: evaluated in t it has no FP32 cancellation.
__device__ __forceinline__ float pp_weight(int r2, const PPParams& P) {
    const float u2 = (float)r2;                   // exact: r2 < 2^24
    const float inv_u = rsqrtf(u2);
    const float x = u2 * inv_u * P.two_over;
    float R;
    if (x <= 1.0f) {
        R = 140.0f - x * x * x * (224.0f + x * x * (-224.0f + x * (70.0f + x * (48.0f - 21.0f * x))));
    } else {
        const float t = 2.0f - x, t2 = t * t;
        R = t2 * t2 * t * (168.0f + t * (-182.0f + t * (64.0f - 7.0f * t)));
    }
    return R * inv_u * inv_u * inv_u;
}

// partner loop of one neighbour cell: accumulate the pair accelerations of the
// particles [q0, q1) whose cell sits dx, dy, dz coarse cells away; pos(q)
// gives their three position bytes
template <class Pos>
__device__ __forceinline__ void pp_cell(int q0, int q1, int dx, int dy, int dz, const int m[3], const PPParams& P,
                                        Pos pos, float& a0, float& a1, float& a2) {
    for (int q = q0; q < q1; ++q) {
        int mq[3];
        pos(q, mq);
        const int sx = 256 * dx + mq[0] - m[0];
        const int sy = 256 * dy + mq[1] - m[1];
        const int sz = 256 * dz + mq[2] - m[2];
        const v2i16 xy = {(short)sx, (short)sy};
        const int r2 = __builtin_amdgcn_sdot2(xy, xy, sz * sz, false);
        if (r2 == 0 || r2 >= P.reach2) continue;
        const float w = pp_weight(r2, P);
        a0 += w * (float)sx;
        a1 += w * (float)sy;
        a2 += w * (float)sz;
    }
}

// Dynamic LDS: own row offsets [Tc + 1], per neighbour row the LDS ranges of
// its Tc + 2 cells [9][Tc + 3], and up to kPPCap packed positions.
__global__ __launch_bounds__(kPPThreads) void k_pp(Geom g, const int32_t* __restrict__ offsets, Planes in,
                                                  float* __restrict__ ax_out, float* __restrict__ ay_out,
                                                  float* __restrict__ az_out, PPParams P) {
    extern __shared__ int lds[];
    const int Tc = g.Tc, RW = Tc + 3;
    int* offs = lds;
    int* s_off = offs + (Tc + 1);
    uint32_t* s_pos = reinterpret_cast<uint32_t*>(s_off + 9 * RW);
    // per neighbour row (dy, dz) = (r % 3 - 1, r / 3 - 1): its first middle
    // cell and the global particle ranges of the middle cells and of the
    // cells just left and right of them
    __shared__ int64_t s_cm[9];
    __shared__ int s_rng[9][6];
    __shared__ int s_base[10];
    const Chunk ch = chunk_of(g, blockIdx.x);
    const int Nc = g.Nc;
    for (int j = threadIdx.x; j <= Tc; j += blockDim.x) offs[j] = offsets[ch.c0 + j];
    if (threadIdx.x < 9) {
        const int r = threadIdx.x;
        const int y = wrapi(ch.cy + r % 3 - 1, Nc), z = wrapi(ch.cz + r / 3 - 1, Nc);
        const int64_t cm = canon(g, ch.cx0, y, z);      // Tc consecutive cells from here
        const int64_t cl = canon(g, wrapi(ch.cx0 - 1, Nc), y, z);
        const int64_t cr = canon(g, wrapi(ch.cx0 + Tc, Nc), y, z);
        s_cm[r] = cm;
        s_rng[r][0] = offsets[cm];
        s_rng[r][1] = offsets[cm + Tc];
        s_rng[r][2] = offsets[cl];
        s_rng[r][3] = offsets[cl + 1];
        s_rng[r][4] = offsets[cr];
        s_rng[r][5] = offsets[cr + 1];
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        int b = 0;
        for (int r = 0; r < 9; ++r) {
            s_base[r] = b;
            b += (s_rng[r][3] - s_rng[r][2]) + (s_rng[r][1] - s_rng[r][0]) + (s_rng[r][5] - s_rng[r][4]);
        }
        s_base[9] = b;
    }
    __syncthreads();
    const bool staged = s_base[9] <= kPPCap;             // uniform over the workgroup
    if (staged) {
        // LDS order per row: left cell, middle cells, right cell
        for (int e = threadIdx.x; e < 9 * RW; e += blockDim.x) {
            const int r = e / RW, i = e - r * RW;
            const int nl = s_rng[r][3] - s_rng[r][2];
            int v;
            if (i == 0)
                v = s_base[r];
            else if (i <= Tc + 1)
                v = s_base[r] + nl + (offsets[s_cm[r] + (i - 1)] - s_rng[r][0]);
            else
                v = s_base[r + 1];
            s_off[e] = v;
        }
        for (int r = 0; r < 9; ++r) {
            const int nl = s_rng[r][3] - s_rng[r][2], nm = s_rng[r][1] - s_rng[r][0];
            const int n = s_base[r + 1] - s_base[r];
            for (int k = threadIdx.x; k < n; k += blockDim.x) {
                const int q = k < nl ? s_rng[r][2] + k : k < nl + nm ? s_rng[r][0] + (k - nl) : s_rng[r][4] + (k - nl - nm);
                s_pos[s_base[r] + k] = (uint32_t)in.m[0][q] | ((uint32_t)in.m[1][q] << 8) | ((uint32_t)in.m[2][q] << 16);
            }
        }
    }
    __syncthreads();
    for (int p = offs[0] + threadIdx.x; p < offs[Tc]; p += blockDim.x) {
        const int j = find_cell(offs, Tc, p);
        const int c[3] = {ch.cx0 + j, ch.cy, ch.cz};
        int m[3], lo[3], hi[3];
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            m[k] = in.m[k][p];
            lo[k] = m[k] < P.reach ? -1 : 0;            // the sphere crosses the lower face
            hi[k] = m[k] + P.reach > 255 ? 1 : 0;       // ... the upper face
        }
        float a0 = 0.0f, a1 = 0.0f, a2 = 0.0f;
        for (int dz = lo[2]; dz <= hi[2]; ++dz) {
            for (int dy = lo[1]; dy <= hi[1]; ++dy) {
                const int r = (dz + 1) * 3 + (dy + 1);
                for (int dx = lo[0]; dx <= hi[0]; ++dx) {
                    if (staged) {
                        const int i = r * RW + j + 1 + dx;
                        pp_cell(s_off[i], s_off[i + 1], dx, dy, dz, m, P,
                                [&](int q, int* mq) {
                                    const uint32_t w = s_pos[q];
                                    mq[0] = (int)(w & 255u);
                                    mq[1] = (int)((w >> 8) & 255u);
                                    mq[2] = (int)(w >> 16);
                                },
                                a0, a1, a2);
                    } else {
                        const int64_t cn = canon(g, wrapi(c[0] + dx, Nc), wrapi(c[1] + dy, Nc), wrapi(c[2] + dz, Nc));
                        pp_cell(offsets[cn], offsets[cn + 1], dx, dy, dz, m, P,
                                [&](int q, int* mq) {
                                    mq[0] = in.m[0][q];
                                    mq[1] = in.m[1][q];
                                    mq[2] = in.m[2][q];
                                },
                                a0, a1, a2);
                    }
                }
            }
        }
        ax_out[p] = a0 * P.amp;
        ay_out[p] = a1 * P.amp;
        az_out[p] = a2 * P.amp;
    }
}

}  // namespace

void launch_pp(const Geom& g, const int32_t* offsets, Planes in, float* const acc[3], hipStream_t s) {
    PPParams P;
    P.reach = 256 * g.npp / g.r;
    P.reach2 = P.reach * P.reach;
    P.two_over = 2.0f / (float)P.reach;
    const double q_per_spacing = 256.0 * g.f / g.r;          // 256 / H
    P.amp = (float)(q_per_spacing * q_per_spacing / (4.0 * M_PI * 140.0));
    const int64_t chunks = g.ncells / g.Tc;
    const size_t lds = sizeof(int) * ((size_t)(g.Tc + 1) + 9 * (size_t)(g.Tc + 3) + kPPCap);
    hipLaunchKernelGGL(k_pp, dim3((unsigned)chunks), dim3(kPPThreads), lds, s, g, offsets, in, acc[0], acc[1], acc[2],
                       P);
}

}  // namespace cube
