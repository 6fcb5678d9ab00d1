// 3-D complex FFTs for the PM Poisson solves (Sec. II, Eq. (1): the force is
// a Fourier-space product of the density and a kernel; Sec. IV names MKL FFT
// for the CPU code -- here every transform is an LDS kernel for gfx950).
//
// Design: each workgroup loads W pencils of length N along one axis into LDS
// (x: W contiguous rows; y, z: W adjacent x-columns, so every global access is
// a run of W*8 contiguous bytes), runs a self-sorting Stockham transform with
// radices 2,3,4,5,7,8 in LDS, and writes back.  Twiddles come from a table of
// exp(-2 pi i k / N) computed in FP64 and rounded once to FP32.  The z pass
// can fuse forward transform, multiplication by a real even Green's table
// (stored as one octant) and inverse transform, so a Poisson solve is five
// sweeps over the mesh: x, y, z+G+z^-1, y^-1, x^-1.
//
// Conventions: forward uses exp(-2 pi i jk/N) like numpy; inverse is
// unnormalised (the 1/N^3 is folded into the Green's tables).
#include <algorithm>
#include <cmath>
#include <vector>

#include "common.h"

namespace cube {

namespace {

constexpr int kFftThreads = 256;

__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ float2 cscale(float2 a, float s) { return make_float2(a.x * s, a.y * s); }
__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
    return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ float2 cmulc(float2 a, float2 b) {   // a * conj(b)
    return make_float2(a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y);
}
// J(a): multiply by -i (forward) or +i (inverse)
template <bool INV>
__device__ __forceinline__ float2 mul_j(float2 a) {
    return INV ? make_float2(-a.y, a.x) : make_float2(a.y, -a.x);
}

// ---- small DFTs in registers --------------------------------------------
template <int R, bool INV>
struct Dft;

template <bool INV>
struct Dft<2, INV> {
    __device__ __forceinline__ static void run(float2* a) {
        float2 t = a[0];
        a[0] = cadd(t, a[1]);
        a[1] = csub(t, a[1]);
    }
};

template <bool INV>
struct Dft<3, INV> {
    __device__ __forceinline__ static void run(float2* a) {
        const float s3 = 0.86602540378443864676f;
        float2 t = cadd(a[1], a[2]);
        float2 m = csub(a[0], cscale(t, 0.5f));
        float2 d = cscale(mul_j<INV>(csub(a[1], a[2])), s3);
        a[0] = cadd(a[0], t);
        a[1] = cadd(m, d);
        a[2] = csub(m, d);
    }
};

template <bool INV>
struct Dft<4, INV> {
    __device__ __forceinline__ static void run(float2* a) {
        float2 t0 = cadd(a[0], a[2]), t1 = csub(a[0], a[2]);
        float2 t2 = cadd(a[1], a[3]), t3 = mul_j<INV>(csub(a[1], a[3]));
        a[0] = cadd(t0, t2);
        a[2] = csub(t0, t2);
        a[1] = cadd(t1, t3);
        a[3] = csub(t1, t3);
    }
};

template <bool INV>
struct Dft<5, INV> {
    __device__ __forceinline__ static void run(float2* a) {
        const float c1 = 0.30901699437494742410f, c2 = -0.80901699437494742410f;
        const float s1 = 0.95105651629515357212f, s2 = 0.58778525229247312917f;
        float2 b1 = cadd(a[1], a[4]), b2 = cadd(a[2], a[3]);
        float2 d1 = csub(a[1], a[4]), d2 = csub(a[2], a[3]);
        float2 r1 = make_float2(a[0].x + c1 * b1.x + c2 * b2.x, a[0].y + c1 * b1.y + c2 * b2.y);
        float2 r2 = make_float2(a[0].x + c2 * b1.x + c1 * b2.x, a[0].y + c2 * b1.y + c1 * b2.y);
        float2 i1 = mul_j<INV>(make_float2(s1 * d1.x + s2 * d2.x, s1 * d1.y + s2 * d2.y));
        float2 i2 = mul_j<INV>(make_float2(s2 * d1.x - s1 * d2.x, s2 * d1.y - s1 * d2.y));
        a[0] = cadd(a[0], cadd(b1, b2));
        a[1] = cadd(r1, i1);
        a[4] = csub(r1, i1);
        a[2] = cadd(r2, i2);
        a[3] = csub(r2, i2);
    }
};

template <bool INV>
struct Dft<7, INV> {
    __device__ __forceinline__ static void run(float2* a) {
        const float c1 = 0.62348980185873353053f, c2 = -0.22252093395631440429f, c3 = -0.90096886790241912624f;
        const float s1 = 0.78183148246802980871f, s2 = 0.97492791218182360702f, s3 = 0.43388373911755812048f;
        float2 b1 = cadd(a[1], a[6]), b2 = cadd(a[2], a[5]), b3 = cadd(a[3], a[4]);
        float2 d1 = csub(a[1], a[6]), d2 = csub(a[2], a[5]), d3 = csub(a[3], a[4]);
        float2 x0 = a[0];
        float2 r1 = make_float2(x0.x + c1 * b1.x + c2 * b2.x + c3 * b3.x, x0.y + c1 * b1.y + c2 * b2.y + c3 * b3.y);
        float2 r2 = make_float2(x0.x + c2 * b1.x + c3 * b2.x + c1 * b3.x, x0.y + c2 * b1.y + c3 * b2.y + c1 * b3.y);
        float2 r3 = make_float2(x0.x + c3 * b1.x + c1 * b2.x + c2 * b3.x, x0.y + c3 * b1.y + c1 * b2.y + c2 * b3.y);
        float2 i1 = mul_j<INV>(make_float2(s1 * d1.x + s2 * d2.x + s3 * d3.x, s1 * d1.y + s2 * d2.y + s3 * d3.y));
        float2 i2 = mul_j<INV>(make_float2(s2 * d1.x - s3 * d2.x - s1 * d3.x, s2 * d1.y - s3 * d2.y - s1 * d3.y));
        float2 i3 = mul_j<INV>(make_float2(s3 * d1.x - s1 * d2.x + s2 * d3.x, s3 * d1.y - s1 * d2.y + s2 * d3.y));
        a[0] = cadd(x0, cadd(b1, cadd(b2, b3)));
        a[1] = cadd(r1, i1);
        a[6] = csub(r1, i1);
        a[2] = cadd(r2, i2);
        a[5] = csub(r2, i2);
        a[3] = cadd(r3, i3);
        a[4] = csub(r3, i3);
    }
};

template <bool INV>
struct Dft<8, INV> {
    __device__ __forceinline__ static void run(float2* a) {
        const float c = 0.70710678118654752440f;
        float2 e[4] = {a[0], a[2], a[4], a[6]};
        float2 o[4] = {a[1], a[3], a[5], a[7]};
        Dft<4, INV>::run(e);
        Dft<4, INV>::run(o);
        // w^1 = (1 -+ i)/sqrt2, w^2 = -+i, w^3 = (-1 -+ i)/sqrt2
        float2 w1 = INV ? make_float2(c * (o[1].x - o[1].y), c * (o[1].x + o[1].y))
                        : make_float2(c * (o[1].x + o[1].y), c * (o[1].y - o[1].x));
        float2 w2 = mul_j<INV>(o[2]);
        float2 w3 = INV ? make_float2(-c * (o[3].x + o[3].y), c * (o[3].x - o[3].y))
                        : make_float2(c * (o[3].y - o[3].x), -c * (o[3].x + o[3].y));
        a[0] = cadd(e[0], o[0]);
        a[4] = csub(e[0], o[0]);
        a[1] = cadd(e[1], w1);
        a[5] = csub(e[1], w1);
        a[2] = cadd(e[2], w2);
        a[6] = csub(e[2], w2);
        a[3] = cadd(e[3], w3);
        a[7] = csub(e[3], w3);
    }
};

// e^{-+2 pi i m / n} for the internal twiddles of the composite DFTs below
// (forward: exp(-2 pi i m / n); inverse: the conjugate)
template <bool INV>
__device__ __forceinline__ float2 rot(float2 a, float c, float s) {
    return INV ? make_float2(a.x * c - a.y * s, a.x * s + a.y * c) : make_float2(a.x * c + a.y * s, a.y * c - a.x * s);
}

// 16 = 4 x 4: DFT-4 over n1 (n = n2 + 4 n1), twiddle w16^(n2 k1), DFT-4 over n2;
// output index k1 + 4 k2
template <bool INV>
struct Dft<16, INV> {
    __device__ __forceinline__ static void run(float2* a) {
        const float c1 = 0.92387953251128675613f, s1 = 0.38268343236508977173f;   // cos, sin(pi/8)
        const float c2 = 0.70710678118654752440f;                                 // cos(pi/4)
        float2 t[4][4];
#pragma unroll
        for (int n2 = 0; n2 < 4; ++n2) {
            float2 v[4] = {a[n2], a[n2 + 4], a[n2 + 8], a[n2 + 12]};
            Dft<4, INV>::run(v);
#pragma unroll
            for (int k1 = 0; k1 < 4; ++k1) t[n2][k1] = v[k1];
        }
        // w16^m for m = n2 k1: 1 (m=0), (c1,s1) m=1, (c2,c2) m=2, (s1,c1) m=3,
        // -i m=4, (-c2,c2) m=6, (-c1,-s1) m=9
        t[1][1] = rot<INV>(t[1][1], c1, s1);
        t[1][2] = rot<INV>(t[1][2], c2, c2);
        t[1][3] = rot<INV>(t[1][3], s1, c1);
        t[2][1] = rot<INV>(t[2][1], c2, c2);
        t[2][2] = mul_j<INV>(t[2][2]);
        t[2][3] = rot<INV>(t[2][3], -c2, c2);
        t[3][1] = rot<INV>(t[3][1], s1, c1);
        t[3][2] = rot<INV>(t[3][2], -c2, c2);
        t[3][3] = rot<INV>(t[3][3], -c1, -s1);
#pragma unroll
        for (int k1 = 0; k1 < 4; ++k1) {
            float2 v[4] = {t[0][k1], t[1][k1], t[2][k1], t[3][k1]};
            Dft<4, INV>::run(v);
#pragma unroll
            for (int k2 = 0; k2 < 4; ++k2) a[k1 + 4 * k2] = v[k2];
        }
    }
};

// 10 = 2 x 5: DFT-5 over n2 (n = n1 + 2 n2), twiddle w10^(n1 k2), DFT-2 over
// n1; output index k2 + 5 k1
template <bool INV>
struct Dft<10, INV> {
    __device__ __forceinline__ static void run(float2* a) {
        const float c36 = 0.80901699437494742410f, s36 = 0.58778525229247312917f;
        const float c72 = 0.30901699437494742410f, s72 = 0.95105651629515357212f;
        float2 e[5] = {a[0], a[2], a[4], a[6], a[8]};
        float2 o[5] = {a[1], a[3], a[5], a[7], a[9]};
        Dft<5, INV>::run(e);
        Dft<5, INV>::run(o);
        // w10^k2 for k2 = 1..4: (cos, sin) of 36, 72, 108, 144 degrees
        o[1] = rot<INV>(o[1], c36, s36);
        o[2] = rot<INV>(o[2], c72, s72);
        o[3] = rot<INV>(o[3], -c72, s72);
        o[4] = rot<INV>(o[4], -c36, s36);
#pragma unroll
        for (int k2 = 0; k2 < 5; ++k2) {
            a[k2] = cadd(e[k2], o[k2]);
            a[k2 + 5] = csub(e[k2], o[k2]);
        }
    }
};

// ---- one Stockham pass over P pencils in LDS -----------------------------
// Layout L: P pencils, element i of pencil w at lds[w*SP + i*SE]; with WFAST
// consecutive threads take consecutive pencils (strided pencils), otherwise
// consecutive butterflies of one pencil (contiguous pencils), so that lanes
// touch consecutive LDS words either way.  NS = product of the radices of
// the passes already done.  WAVE: the pencils belong to one wave (NT = 64),
// which synchronises only with itself, so the waves of a workgroup need not
// run their passes in step; the first npen of the P pencils are live.
template <int P_, int SE_, int SP_, bool WFAST_, int NT_, bool WAVE_ = false>
struct Lay {
    static constexpr int P = P_, SE = SE_, SP = SP_, NT = NT_;
    static constexpr bool WFAST = WFAST_, WAVE = WAVE_;
};

// LDS ordering among the lanes of one wave: its LDS operations complete in
// issue order, so it is enough to keep the compiler from moving them across
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <class L>
__device__ __forceinline__ void lay_sync() {
    if (L::WAVE) wave_sync();
    else lds_barrier();
}

template <int N, class L, bool INV, int NS, int R>
__device__ __forceinline__ void stockham_pass(float2* lds, const float2* __restrict__ tw, int tid, int npen) {
    constexpr int NB = N / R;
    constexpr int TOTAL = NB * L::P;
    constexpr int IT = (TOTAL + L::NT - 1) / L::NT;
    float2 v[IT][R];
#pragma unroll
    for (int it = 0; it < IT; ++it) {
        const int b = tid + it * L::NT;
        const int j = L::WFAST ? b / L::P : b % NB;
        const int w = L::WFAST ? b % L::P : b / NB;
        if ((TOTAL % L::NT == 0 || b < TOTAL) && (!L::WAVE || w < npen)) {
            const float2* col = lds + w * L::SP;
#pragma unroll
            for (int r = 0; r < R; ++r) v[it][r] = col[(j + r * NB) * L::SE];
            if (NS > 1) {
                const int k = j % NS;
#pragma unroll
                for (int r = 1; r < R; ++r) {
                    const float2 t = tw[(r * k) * (N / (NS * R))];
                    v[it][r] = INV ? cmulc(v[it][r], t) : cmul(v[it][r], t);
                }
            }
            Dft<R, INV>::run(v[it]);
        }
    }
    lay_sync<L>();
#pragma unroll
    for (int it = 0; it < IT; ++it) {
        const int b = tid + it * L::NT;
        const int j = L::WFAST ? b / L::P : b % NB;
        const int w = L::WFAST ? b % L::P : b / NB;
        if ((TOTAL % L::NT == 0 || b < TOTAL) && (!L::WAVE || w < npen)) {
            const int k = j % NS;
            float2* col = lds + w * L::SP + ((j / NS) * NS * R + k) * L::SE;
#pragma unroll
            for (int r = 0; r < R; ++r) col[r * NS * L::SE] = v[it][r];
        }
    }
    lay_sync<L>();
}

template <int N, class L, bool INV, int NS>
__device__ __forceinline__ void run_passes(float2*, const float2*, int, int) {}

template <int N, class L, bool INV, int NS, int R, int... Rest>
__device__ __forceinline__ void run_passes(float2* lds, const float2* __restrict__ tw, int tid, int npen) {
    stockham_pass<N, L, INV, NS, R>(lds, tw, tid, npen);
    run_passes<N, L, INV, NS * R, Rest...>(lds, tw, tid, npen);
}

// Radix plan per supported size.
template <int N>
struct Plan;
#define CUBE_FFT_PLAN(NN, ...)                                                   \
    template <>                                                                  \
    struct Plan<NN> {                                                            \
        template <class L, bool INV>                                             \
        __device__ __forceinline__ static void run(float2* lds,                  \
                                                   const float2* __restrict__ tw, \
                                                   int tid = threadIdx.x,        \
                                                   int npen = L::P) {            \
            run_passes<NN, L, INV, 1, __VA_ARGS__>(lds, tw, tid, npen);          \
        }                                                                        \
    };
CUBE_FFT_PLAN(16, 4, 4)
CUBE_FFT_PLAN(32, 4, 8)
CUBE_FFT_PLAN(48, 3, 4, 4)
CUBE_FFT_PLAN(64, 8, 8)
CUBE_FFT_PLAN(80, 5, 4, 4)
CUBE_FFT_PLAN(96, 3, 4, 8)
CUBE_FFT_PLAN(112, 7, 4, 4)
CUBE_FFT_PLAN(128, 2, 8, 8)
CUBE_FFT_PLAN(160, 10, 16)
CUBE_FFT_PLAN(192, 3, 8, 8)
CUBE_FFT_PLAN(224, 7, 4, 8)
CUBE_FFT_PLAN(256, 4, 8, 8)
CUBE_FFT_PLAN(320, 5, 8, 8)
CUBE_FFT_PLAN(384, 3, 2, 8, 8)
CUBE_FFT_PLAN(448, 7, 8, 8)
CUBE_FFT_PLAN(512, 8, 8, 8)
CUBE_FFT_PLAN(1024, 4, 4, 8, 8)
#undef CUBE_FFT_PLAN

// Plan of the z-pencil pass (16 pencils per 256-thread workgroup): the same
// radices.  At N = 160 the 10 x 16 plan takes one radix-10 and 5/8 of a
// radix-16 butterfly per thread and crosses LDS once less than 5, 4, 8 with
// every thread busy (31.7 against 33.7 ms per 1024^3 step).
template <int N>
struct PlanZ : Plan<N> {};

template <int N>
constexpr int pencils() { return N <= 256 ? 16 : 8; }

__device__ __forceinline__ int fold(int k, int n) { return k <= n / 2 ? k : n - k; }

// KIND: 0 = x pencils, 1 = y pencils, 2 = z pencils.
// MODE: 0 forward, 1 inverse, 2 forward * float table * inverse, 3 same with a double table.
template <int N, int KIND, int MODE>
__global__ __launch_bounds__(kFftThreads) void k_fft(float2* __restrict__ data, const float2* __restrict__ tw,
                                                      const void* __restrict__ green) {
    constexpr int W = pencils<N>();
    constexpr int LDN = N + 1;
    __shared__ float2 lds[W * LDN];
    float2* cube_base = data + (int64_t)blockIdx.y * N * N * N;
    const int b = blockIdx.x;
    int64_t base;
    int64_t stride_i, stride_w;
    int x0 = 0, yz = 0;
    if (KIND == 0) {            // rows b*W .. b*W+W-1, each N contiguous
        base = (int64_t)b * W * N;
        stride_i = 1;
        stride_w = N;
    } else {
        x0 = (b % (N / W)) * W;
        yz = b / (N / W);
        stride_w = 1;
        if (KIND == 1) {        // along y at fixed z
            base = x0 + (int64_t)N * N * yz;
            stride_i = N;
        } else {                // along z at fixed y
            base = x0 + (int64_t)N * yz;
            stride_i = (int64_t)N * N;
        }
    }
    float2* g = cube_base + base;
    stage_to_lds<kFftThreads, 8>(
        W * N, g, lds,
        [&](int e) {
            const int i = KIND == 0 ? e % N : e / W, w = KIND == 0 ? e / N : e % W;
            return (int64_t)i * stride_i + (int64_t)w * stride_w;
        },
        [&](int e) {
            const int i = KIND == 0 ? e % N : e / W, w = KIND == 0 ? e / N : e % W;
            return w * LDN + i;
        });
    lds_barrier();
    using L = Lay<W, 1, LDN, false, kFftThreads>;
    if (MODE == 1) {
        Plan<N>::template run<L, true>(lds, tw);
    } else {
        Plan<N>::template run<L, false>(lds, tw);
    }
    if (MODE >= 2) {
        // multiply by G(kx, ky, kz): this block holds kz = i, ky = yz, kx = x0 + w
        constexpr int M = N / 2 + 1;
        const int fy = fold(yz, N);
        for (int e = threadIdx.x; e < W * N; e += kFftThreads) {
            const int w = e % W, i = e / W;
            const int64_t gi = ((int64_t)fold(i, N) * M + fy) * M + fold(x0 + w, N);
            float2 v = lds[w * LDN + i];
            if (MODE == 2) {
                const float gv = static_cast<const float*>(green)[gi];
                v = make_float2(v.x * gv, v.y * gv);
            } else {
                const double gv = static_cast<const double*>(green)[gi];
                v = make_float2((float)((double)v.x * gv), (float)((double)v.y * gv));
            }
            lds[w * LDN + i] = v;
        }
        lds_barrier();
        Plan<N>::template run<L, true>(lds, tw);
    }
    for (int e = threadIdx.x; e < W * N; e += kFftThreads) {
        int i, w;
        if (KIND == 0) { i = e % N; w = e / N; } else { w = e % W; i = e / W; }
        g[i * stride_i + w * stride_w] = lds[w * LDN + i];
    }
}

// ---- storage of the half spectra between the tile sweeps ----------------
// FP32 complex, or one 32-bit word with two 16-bit values (real part in the
// low half).  BF16 is rounded to nearest even from FP32 and needs no scaling;
// FP16 values are stored times a power of two chosen by the host so that the
// spectra of realistic densities and potentials stay inside its range, and
// any value that would not fit raises the caller's flag.
enum SpecFmt { SPEC_F32 = 0, SPEC_BF16 = 1, SPEC_F16 = 2 };

template <int FMT>
struct SpecStore;

template <>
struct SpecStore<SPEC_F32> {
    using T = float2;
    __device__ __forceinline__ static float2 get(T v, float) { return v; }
    __device__ __forceinline__ static T put(float2 v, float, bool&) { return v; }
};

template <>
struct SpecStore<SPEC_BF16> {
    using T = uint32_t;
    __device__ __forceinline__ static float2 get(T v, float) {
        return make_float2(__uint_as_float(v << 16), __uint_as_float(v & 0xffff0000u));
    }
    __device__ __forceinline__ static uint32_t bf16(float x) {
        const uint32_t b = __float_as_uint(x);
        return (b + 0x7fffu + ((b >> 16) & 1u)) >> 16;
    }
    __device__ __forceinline__ static T put(float2 v, float, bool&) { return bf16(v.x) | (bf16(v.y) << 16); }
};

template <>
struct SpecStore<SPEC_F16> {
    using T = uint32_t;
    __device__ __forceinline__ static float h2f(uint32_t bits) {
        return (float)__builtin_bit_cast(_Float16, (uint16_t)bits);
    }
    __device__ __forceinline__ static uint32_t f2h(float x) { return __builtin_bit_cast(uint16_t, (_Float16)x); }
    __device__ __forceinline__ static float2 get(T v, float scale) {
        return make_float2(h2f(v & 0xffffu) * scale, h2f(v >> 16) * scale);
    }
    __device__ __forceinline__ static T put(float2 v, float scale, bool& bad) {
        const float a = v.x * scale, b = v.y * scale;
        bad = bad || !(fabsf(a) <= 65504.0f) || !(fabsf(b) <= 65504.0f);
        return f2h(a) | (f2h(b) << 16);
    }
};

__device__ __forceinline__ void raise_flag(bool bad, int32_t* flag) {
    if (bad) *flag = 1;
}

// ---- real tile meshes: R2C / C2R through xy planes ---------------------
// A tile's real mesh [z][y][x] (N^3 floats) maps to a half spectrum
// [kz][ky][kx], kx in [0, N/2] (N^2 (N/2+1) complex).  One workgroup owns a
// whole z-plane in LDS: rows 2j and 2j+1 are transformed together as one
// complex row and separated with the Hermitian symmetry, then the N/2+1
// columns are transformed along y.  The inverse runs the same steps backwards.
constexpr int kPlaneThreads = 1024;

// Persistent: each workgroup walks planes blockIdx.x, +gridDim.x, ...; the
// next plane's global loads are issued into registers before the current
// plane's LDS passes, so memory and LDS work overlap even at one workgroup
// per CU.  Twiddles live in LDS so no global load sits inside the passes.
// Complex row j (real rows 2j, 2j+1) sits at lds[j*(N+2) + x], which is also
// where the separated half-spectrum rows 2j and 2j+1 (stride N/2+1) go, so
// the Hermitian separation is done row by row in place, one wave per row:
// a wave's LDS reads all complete before its writes.
template <int N, int FMT>
__global__ __launch_bounds__(kPlaneThreads) void k_r2c_plane(const float* __restrict__ real_tiles,
                                                             typename SpecStore<FMT>::T* __restrict__ spec_tiles,
                                                             const float2* __restrict__ tw_g, int nplanes,
                                                             float sc_out, int32_t* __restrict__ flag) {
    using S = SpecStore<FMT>;
    constexpr int NH = N / 2 + 1;
    constexpr int HALF = N / 2;
    constexpr int RS = N + 2;                    // complex row stride = 2 NH
    constexpr int TOT = HALF * N;
    constexpr int PER = (TOT + kPlaneThreads - 1) / kPlaneThreads;
    constexpr int KIT = (NH + kWave - 1) / kWave;
    constexpr int NW = kPlaneThreads / kWave;
    __shared__ float2 lds[HALF * RS];
    __shared__ float2 tw[N];
    for (int i = threadIdx.x; i < N; i += kPlaneThreads) tw[i] = tw_g[i];
    const int lane = threadIdx.x & (kWave - 1), wv = threadIdx.x / kWave;
    float re[PER], im[PER];
    auto prefetch = [&](int pl) {
        const float* src = real_tiles + (int64_t)(pl / N) * N * N * N + (int64_t)(pl % N) * N * N;
#pragma unroll
        for (int u = 0; u < PER; ++u) {
            const int e = threadIdx.x + u * kPlaneThreads;
            if (TOT % kPlaneThreads == 0 || e < TOT) {
                const int j = e / N, x = e % N;
                re[u] = src[(2 * j) * N + x];
                im[u] = src[(2 * j + 1) * N + x];
            }
        }
    };
    int plane = blockIdx.x;
    if (plane < nplanes) prefetch(plane);
    for (; plane < nplanes; plane += gridDim.x) {
        lds_barrier();
#pragma unroll
        for (int u = 0; u < PER; ++u) {
            const int e = threadIdx.x + u * kPlaneThreads;
            if (TOT % kPlaneThreads == 0 || e < TOT) lds[(e / N) * RS + e % N] = make_float2(re[u], im[u]);
        }
        lds_barrier();
        if (plane + (int)gridDim.x < nplanes) prefetch(plane + gridDim.x);
        // a fresh, opaque thread index per plane keeps the passes' LDS
        // address arithmetic from being hoisted out of the plane loop
        int tid = threadIdx.x;
        asm volatile("" : "+v"(tid));
        Plan<N>::template run<Lay<HALF, 1, RS, false, kPlaneThreads>, false>(lds, tw, tid);
        // A(k) = (Z(k) + conj Z(N-k)) / 2, B(k) = (Z(k) - conj Z(N-k)) / 2i, k = 0..N/2
        for (int j = wv; j < HALF; j += NW) {
            float2* row = lds + j * RS;
            float2 va[KIT], vb[KIT];
#pragma unroll
            for (int t = 0; t < KIT; ++t) {
                const int k = lane + t * kWave;
                if (k < NH) {
                    const float2 z1 = row[k];
                    const float2 z2 = row[k == 0 ? 0 : N - k];
                    va[t] = make_float2(0.5f * (z1.x + z2.x), 0.5f * (z1.y - z2.y));
                    vb[t] = make_float2(0.5f * (z1.y + z2.y), 0.5f * (z2.x - z1.x));
                }
            }
            __builtin_amdgcn_wave_barrier();
#pragma unroll
            for (int t = 0; t < KIT; ++t) {
                const int k = lane + t * kWave;
                if (k < NH) {
                    row[k] = va[t];
                    row[NH + k] = vb[t];
                }
            }
        }
        lds_barrier();
        Plan<N>::template run<Lay<NH, NH, 1, true, kPlaneThreads>, false>(lds, tw, tid);
        typename S::T* dst = spec_tiles + (int64_t)(plane / N) * N * N * NH + (int64_t)(plane % N) * N * NH;
        bool bad = false;
        for (int e = threadIdx.x; e < N * NH; e += kPlaneThreads) dst[e] = S::put(lds[e], sc_out, bad);
        if (FMT == SPEC_F16) raise_flag(bad, flag);
    }
}

template <int N, int FMT>
__global__ __launch_bounds__(kPlaneThreads) void k_c2r_plane(const typename SpecStore<FMT>::T* __restrict__ spec_tiles,
                                                             float* __restrict__ real_tiles,
                                                             const float2* __restrict__ tw_g, int nplanes,
                                                             float sc_in, int lo, int hi) {
    using S = SpecStore<FMT>;
    constexpr int NH = N / 2 + 1;
    constexpr int HALF = N / 2;
    constexpr int RS = N + 2;
    constexpr int TOT = N * NH;
    // only the window [lo, hi)^3 of each tile is produced: planes lo..hi-1,
    // and in each plane the rows and columns lo..hi-1
    const int W = hi - lo;
    const int jlo = lo / 2, jhi = (hi + 1) / 2;
    const int st_y = (int)threadIdx.x / W, st_x = (int)threadIdx.x % W;           // once per thread
    const int step_y = kPlaneThreads / W, step_x = kPlaneThreads % W;
    constexpr int PER = (TOT + kPlaneThreads - 1) / kPlaneThreads;
    constexpr int KIT = (N + kWave - 1) / kWave;
    constexpr int NW = kPlaneThreads / kWave;
    __shared__ float2 lds[HALF * RS];
    __shared__ float2 tw[N];
    for (int i = threadIdx.x; i < N; i += kPlaneThreads) tw[i] = tw_g[i];
    const int lane = threadIdx.x & (kWave - 1), wv = threadIdx.x / kWave;
    typename S::T pv[PER];
    auto prefetch = [&](int pl) {
        const typename S::T* src = spec_tiles + (int64_t)(pl / W) * N * N * NH + (int64_t)(lo + pl % W) * N * NH;
#pragma unroll
        for (int u = 0; u < PER; ++u) {
            const int e = threadIdx.x + u * kPlaneThreads;
            if (TOT % kPlaneThreads == 0 || e < TOT) pv[u] = src[e];
        }
    };
    int plane = blockIdx.x;
    if (plane < nplanes) prefetch(plane);
    for (; plane < nplanes; plane += gridDim.x) {
        lds_barrier();
#pragma unroll
        for (int u = 0; u < PER; ++u) {
            const int e = threadIdx.x + u * kPlaneThreads;
            if (TOT % kPlaneThreads == 0 || e < TOT) lds[e] = S::get(pv[u], sc_in);
        }
        lds_barrier();
        if (plane + (int)gridDim.x < nplanes) prefetch(plane + gridDim.x);
        // a fresh, opaque thread index per plane keeps the passes' LDS
        // address arithmetic from being hoisted out of the plane loop
        int tid = threadIdx.x;
        asm volatile("" : "+v"(tid));
        Plan<N>::template run<Lay<NH, NH, 1, true, kPlaneThreads>, true>(lds, tw, tid);
        // complex row Z(k) = A(k) + i B(k) over k = 0..N-1 (Hermitian extension of A, B)
        for (int j = jlo + wv; j < jhi; j += NW) {
            float2* row = lds + j * RS;
            float2 vz[KIT];
#pragma unroll
            for (int t = 0; t < KIT; ++t) {
                const int k = lane + t * kWave;
                if (k < N) {
                    const int kk = k <= HALF ? k : N - k;
                    const float sg = k <= HALF ? 1.0f : -1.0f;
                    const float2 a = row[kk], b = row[NH + kk];
                    vz[t] = make_float2(a.x - sg * b.y, sg * a.y + b.x);
                }
            }
            __builtin_amdgcn_wave_barrier();
#pragma unroll
            for (int t = 0; t < KIT; ++t) {
                const int k = lane + t * kWave;
                if (k < N) row[k] = vz[t];
            }
        }
        lds_barrier();
        Plan<N>::template run<Lay<HALF, 1, RS, false, kPlaneThreads>, true>(lds, tw, tid);
        float* dst = real_tiles + (int64_t)(plane / W) * N * N * N + (int64_t)(lo + plane % W) * N * N;
        // element e = (y - lo) W + (x - lo), walked with increments instead of divisions
        int y = lo + st_y, x = lo + st_x;
        for (int e = threadIdx.x; e < W * W; e += kPlaneThreads) {
            const float2 v = lds[(y >> 1) * RS + x];
            dst[y * N + x] = (y & 1) ? v.y : v.x;
            x += step_x;
            y += step_y;
            if (x >= hi) {
                x -= W;
                ++y;
            }
        }
    }
}

// Wave-owned variants (N/2 divisible by the 16 waves): wave w owns complex
// rows [w R, (w+1) R), R = N/32, for the row transforms and the Hermitian
// step, and up to C = ceil((N/2+1)/16) columns for the column transforms.
// Inside each phase a wave synchronises only with itself, so one wave's LDS
// traffic overlaps another's arithmetic; the workgroup meets three times per
// plane (plane in LDS, rows done, columns done).  The forward kernel loads
// each wave's own rows from HBM, the inverse one stores each wave's own rows.
// Makes the compiler wait for a register's pending load here.
__device__ __forceinline__ void touch_reg(float2 v) { asm volatile("" ::"v"(v.x), "v"(v.y)); }
__device__ __forceinline__ void touch_reg(uint32_t v) { asm volatile("" ::"v"(v)); }

template <int N>
struct PlaneSplit {
    static constexpr int NW = kPlaneThreads / kWave;
    static constexpr int HALF = N / 2, NH = N / 2 + 1;
    // real row y of the half spectrum sits at y RSH (two per complex row of
    // stride RS = 2 RSH); RSH = NH + 4 makes 2 RS = 20 (mod 64) dwords, so the
    // rows a wave's lanes touch together start in different LDS banks
    static constexpr int RSH = NH % 16 == 1 ? NH + 4 : NH, RS = 2 * RSH;
    static constexpr int RPW = HALF / NW;                  // complex rows per wave
    static constexpr int CPW = (NH + NW - 1) / NW;         // columns per wave (the last waves fewer)
    static constexpr bool ok = HALF % NW == 0;
};

template <int N, int FMT>
__global__ __launch_bounds__(kPlaneThreads) void k_r2c_plane_w(const float* __restrict__ real_tiles,
                                                               typename SpecStore<FMT>::T* __restrict__ spec_tiles,
                                                               const float2* __restrict__ tw_g, int nplanes,
                                                               float sc_out, int32_t* __restrict__ flag) {
    using S = SpecStore<FMT>;
    using PS = PlaneSplit<N>;
    constexpr int NH = PS::NH, RS = PS::RS, RSH = PS::RSH, RPW = PS::RPW, CPW = PS::CPW;
    constexpr int EPW = RPW * N;                             // complex elements of a wave's rows
    constexpr int PER = (EPW + kWave - 1) / kWave;
    constexpr int KIT = (NH + kWave - 1) / kWave;
    __shared__ float2 lds[PS::HALF * RS];
    __shared__ float2 tw[N];
    for (int i = threadIdx.x; i < N; i += kPlaneThreads) tw[i] = tw_g[i];
    const int lane = threadIdx.x & (kWave - 1), wv = threadIdx.x / kWave;
    const int j0 = wv * RPW;
    const int c0 = wv * CPW, ncol = NH - c0 < CPW ? NH - c0 : CPW;
    float re[PER], im[PER];
    // lane indices pass through an opaque copy per use, so that per-element
    // offsets are recomputed each plane instead of held in registers
    auto prefetch = [&](int pl) {
        int ln = lane;
        asm volatile("" : "+v"(ln));
        const float* src = real_tiles + (int64_t)(pl / N) * N * N * N + (int64_t)(pl % N) * N * N + 2 * j0 * N;
        // every lane loads (the last round's idle lanes re-read the wave's
        // last element): branch-free loads keep the wait counts exact
#pragma unroll
        for (int u = 0; u < PER; ++u) {
            int e = ln + u * kWave;
            if ((u + 1) * kWave > EPW) e = e < EPW ? e : EPW - 1;
            const int j = e / N, x = e % N;
            re[u] = src[(2 * j) * N + x];
            im[u] = src[(2 * j + 1) * N + x];
        }
    };
    bool bad = false;
    int plane = blockIdx.x;
    if (plane < nplanes) prefetch(plane);
    // the first plane's loads are waited for here, so that no path into the
    // loop's top has loads pending and the top never waits
#pragma unroll
    for (int u = 0; u < PER; ++u) asm volatile("" ::"v"(re[u]), "v"(im[u]));
    for (; plane < nplanes; plane += gridDim.x) {
        lds_barrier();                                     // the previous plane's spectrum is stored
        float2* rows = lds + j0 * RS;
#pragma unroll
        for (int u = 0; u < PER; ++u) {
            const int e = lane + u * kWave;
            if ((u + 1) * kWave <= EPW || e < EPW) rows[(e / N) * RS + e % N] = make_float2(re[u], im[u]);
        }
        wave_sync();
        if (plane + (int)gridDim.x < nplanes) prefetch(plane + gridDim.x);
        asm volatile("" ::: "memory");                       // keep the prefetch loads here, ahead of the passes
        int tid = lane;
        asm volatile("" : "+v"(tid));
        Plan<N>::template run<Lay<RPW, 1, RS, false, kWave, true>, false>(rows, tw, tid);
        // A(k) = (Z(k) + conj Z(N-k)) / 2, B(k) = (Z(k) - conj Z(N-k)) / 2i, k = 0..N/2
        for (int j = 0; j < RPW; ++j) {
            float2* row = rows + j * RS;
            float2 va[KIT], vb[KIT];
#pragma unroll
            for (int t = 0; t < KIT; ++t) {
                const int k = lane + t * kWave;
                if (k < NH) {
                    const float2 z1 = row[k];
                    const float2 z2 = row[k == 0 ? 0 : N - k];
                    va[t] = make_float2(0.5f * (z1.x + z2.x), 0.5f * (z1.y - z2.y));
                    vb[t] = make_float2(0.5f * (z1.y + z2.y), 0.5f * (z2.x - z1.x));
                }
            }
            wave_sync();
#pragma unroll
            for (int t = 0; t < KIT; ++t) {
                const int k = lane + t * kWave;
                if (k < NH) {
                    row[k] = va[t];
                    row[RSH + k] = vb[t];
                }
            }
            wave_sync();
        }
        lds_barrier();                                     // every row transformed
        if (ncol > 0)
            Plan<N>::template run<Lay<CPW, RSH, 1, true, kWave, true>, false>(lds + c0, tw, tid, ncol);
        lds_barrier();                                     // every column transformed
        // Loads and stores share one in-order counter: wait for the next
        // plane's loads (issued long before, so this costs nothing) ahead of
        // the stores, so that the top of the next iteration does not wait
        // for these stores to complete.
#pragma unroll
        for (int u = 0; u < PER; ++u) asm volatile("" ::"v"(re[u]), "v"(im[u]));
        typename S::T* dst = spec_tiles + (int64_t)(plane / N) * N * N * NH + (int64_t)(plane % N) * N * NH;
        constexpr int SPT = (N * NH + kPlaneThreads - 1) / kPlaneThreads;
        int t = threadIdx.x;
        asm volatile("" : "+v"(t));
#pragma unroll
        for (int u = 0; u < SPT; ++u) {
            const int e = t + u * kPlaneThreads;
            if ((u + 1) * kPlaneThreads <= N * NH || e < N * NH)
                dst[e] = S::put(lds[(e / NH) * RSH + e % NH], sc_out, bad);
        }
    }
    if (FMT == SPEC_F16) raise_flag(bad, flag);
}

template <int N, int FMT>
__global__ __launch_bounds__(kPlaneThreads) void k_c2r_plane_w(const typename SpecStore<FMT>::T* __restrict__ spec_tiles,
                                                               float* __restrict__ real_tiles,
                                                               const float2* __restrict__ tw_g, int nplanes,
                                                               float sc_in, int lo, int hi) {
    using S = SpecStore<FMT>;
    using PS = PlaneSplit<N>;
    constexpr int NH = PS::NH, RS = PS::RS, RSH = PS::RSH, RPW = PS::RPW, CPW = PS::CPW, HALF = PS::HALF;
    constexpr int TOT = N * NH;
    constexpr int PER = (TOT + kPlaneThreads - 1) / kPlaneThreads;
    constexpr int KIT = (N + kWave - 1) / kWave;
    // only the window [lo, hi)^3 of each tile is produced: planes lo..hi-1,
    // and in each plane the rows and columns lo..hi-1
    const int W = hi - lo;
    __shared__ float2 lds[HALF * RS];
    __shared__ float2 tw[N];
    for (int i = threadIdx.x; i < N; i += kPlaneThreads) tw[i] = tw_g[i];
    const int lane = threadIdx.x & (kWave - 1), wv = threadIdx.x / kWave;
    const int j0 = wv * RPW;
    const int c0 = wv * CPW, ncol = NH - c0 < CPW ? NH - c0 : CPW;
    // the wave's real rows [2 j0, 2 j0 + 2 RPW) that fall in the window
    const int ya = 2 * j0 > lo ? 2 * j0 : lo, yb = 2 * (j0 + RPW) < hi ? 2 * (j0 + RPW) : hi;
    const bool rows_live = ya < yb;
    typename S::T pv[PER];
    auto prefetch = [&](int pl) {
        const typename S::T* src = spec_tiles + (int64_t)(pl / W) * N * N * NH + (int64_t)(lo + pl % W) * N * NH;
#pragma unroll
        for (int u = 0; u < PER; ++u) {
            const int e = threadIdx.x + u * kPlaneThreads;
            if (TOT % kPlaneThreads == 0 || e < TOT) pv[u] = src[e];
        }
    };
    int plane = blockIdx.x;
    if (plane < nplanes) prefetch(plane);
    // the first plane's loads are waited for here, so that no path into the
    // loop's top has loads pending and the top never waits
#pragma unroll
    for (int u = 0; u < PER; ++u) touch_reg(pv[u]);
    for (; plane < nplanes; plane += gridDim.x) {
        lds_barrier();                                     // the previous plane's rows are stored
#pragma unroll
        for (int u = 0; u < PER; ++u) {
            const int e = threadIdx.x + u * kPlaneThreads;
            if (TOT % kPlaneThreads == 0 || e < TOT) lds[(e / NH) * RSH + e % NH] = S::get(pv[u], sc_in);
        }
        lds_barrier();                                     // the plane's spectrum is in LDS
        if (plane + (int)gridDim.x < nplanes) prefetch(plane + gridDim.x);
        int tid = lane;
        asm volatile("" : "+v"(tid));
        if (ncol > 0)
            Plan<N>::template run<Lay<CPW, RSH, 1, true, kWave, true>, true>(lds + c0, tw, tid, ncol);
        lds_barrier();                                     // every column transformed
        // Loads and stores share one in-order counter: wait for the next
        // plane's loads (issued long before) ahead of this plane's stores, so
        // that the top of the next iteration does not wait for the stores.
#pragma unroll
        for (int u = 0; u < PER; ++u) touch_reg(pv[u]);
        if (rows_live) {
            float2* rows = lds + j0 * RS;
            // complex row Z(k) = A(k) + i B(k) over k = 0..N-1 (Hermitian extension of A, B)
            for (int j = 0; j < RPW; ++j) {
                float2* row = rows + j * RS;
                float2 vz[KIT];
#pragma unroll
                for (int t = 0; t < KIT; ++t) {
                    const int k = lane + t * kWave;
                    if (k < N) {
                        const int kk = k <= HALF ? k : N - k;
                        const float sg = k <= HALF ? 1.0f : -1.0f;
                        const float2 a = row[kk], b = row[RSH + kk];
                        vz[t] = make_float2(a.x - sg * b.y, sg * a.y + b.x);
                    }
                }
                wave_sync();
#pragma unroll
                for (int t = 0; t < KIT; ++t) {
                    const int k = lane + t * kWave;
                    if (k < N) row[k] = vz[t];
                }
                wave_sync();
            }
            Plan<N>::template run<Lay<RPW, 1, RS, false, kWave, true>, true>(rows, tw, tid);
            float* dst = real_tiles + (int64_t)(plane / W) * N * N * N + (int64_t)(lo + plane % W) * N * N;
            // elements (y, x) of rows [ya, yb), x in [lo, hi), walked with increments
            int y = ya, x = lo + lane;
            while (x >= hi) {
                x -= W;
                ++y;
            }
            while (y < yb) {
                const float2 v = lds[(y >> 1) * RS + x];
                dst[y * N + x] = (y & 1) ? v.y : v.x;
                x += kWave;
                while (x >= hi) {
                    x -= W;
                    ++y;
                }
            }
        }
    }
}

// z pencils of the half spectrum: forward, times G (float octant), inverse.
// Twiddles and the block's Green's values are staged in LDS with the data.
template <int N, int FMT>
__global__ __launch_bounds__(kFftThreads) void k_zconv_half(typename SpecStore<FMT>::T* __restrict__ spec_tiles,
                                                            const float2* __restrict__ tw_g,
                                                            const float* __restrict__ green, float sc_in,
                                                            float sc_out, int32_t* __restrict__ flag, int lo,
                                                            int hi) {
    using S = SpecStore<FMT>;
    using T = typename S::T;
    constexpr int ZT = kFftThreads;
    constexpr int NH = N / 2 + 1;
    constexpr int W = 16;
    constexpr int LDN = N + 1;
    constexpr int PLANE = N * NH;
    constexpr int U = (W * N + ZT - 1) / ZT < 10 ? (W * N + ZT - 1) / ZT : 10;
    __shared__ float2 lds[W * LDN];
    __shared__ float2 tw[N];
    __shared__ float gl[W * NH];                   // G of this block's (ky, kx) pencils, by folded kz
    const int c0 = blockIdx.x * W;                 // flattened (ky, kx) of the first pencil
    T* g = spec_tiles + (int64_t)blockIdx.y * N * PLANE + c0;
    for (int i = threadIdx.x; i < N; i += ZT) tw[i] = tw_g[i];
    // table is pencil-major ([ky][kx][kz], kz fastest): consecutive lanes read
    // consecutive kz of one pencil and keep that order in LDS (gl[w][kz])
    for (int e = threadIdx.x; e < W * NH; e += ZT) {
        const int fz = e % NH, w = e / NH;
        const int c = c0 + w;
        const int ky = c / NH, kx = c - ky * NH;
        gl[e] = green[((int64_t)fold(ky, N) * NH + kx) * NH + fz];
    }
    // element e: pencil w = e % W, kz = e / W (16 consecutive words per kz)
    for (int base = 0; base < W * N; base += ZT * U) {
        T tmp[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int e = base + u * ZT + (int)threadIdx.x;
            if (e < W * N) tmp[u] = g[(int64_t)(e / W) * PLANE + (e % W)];
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int e = base + u * ZT + (int)threadIdx.x;
            if (e < W * N) lds[(e % W) * LDN + e / W] = S::get(tmp[u], sc_in);
        }
    }
    lds_barrier();
    using L = Lay<W, 1, LDN, false, ZT>;
    PlanZ<N>::template run<L, false>(lds, tw);
    for (int e = threadIdx.x; e < W * N; e += ZT) {
        const int w = e % W, i = e / W;
        const float gv = gl[w * NH + fold(i, N)];
        const float2 v = lds[w * LDN + i];
        lds[w * LDN + i] = make_float2(v.x * gv, v.y * gv);
    }
    lds_barrier();
    PlanZ<N>::template run<L, true>(lds, tw);
    bool bad = false;
    for (int e = threadIdx.x; e < W * (hi - lo); e += ZT) {       // only z in [lo, hi) is used
        const int w = e % W, i = lo + e / W;
        g[(int64_t)i * PLANE + w] = S::put(lds[w * LDN + i], sc_out, bad);
    }
    if (FMT == SPEC_F16) raise_flag(bad, flag);
}

int device_cus() {
    static const int cus = [] {
        int dev = 0, v = 0;
        hipGetDevice(&dev);
        if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || v <= 0) v = 256;
        return v;
    }();
    return cus;
}

template <int N, int FMT>
void launch_tiles_fmt(float* real_tiles, void* spec, int ntiles, const float2* tw, const float* green,
                      int32_t* flag, int lo, int hi, hipStream_t s, hipEvent_t* ev) {
    constexpr int NH = N / 2 + 1;
    using T = typename SpecStore<FMT>::T;
    T* spec_tiles = static_cast<T*>(spec);
    // FP16 scales.  The xy-plane spectra of the density are sums of N^2
    // cells: stored times 2^-e with 2^e >= N^2 they stay below max|rho - 1|
    // (the host keeps that inside the FP16 range).  After the z pencils and
    // the Green's multiply (which carries the 1/N^3 of the inverse
    // transform) the values are the normalised 2-D coefficients of the
    // potential, bounded by max|phi| and typically max|phi| / N: stored times
    // 2^5 they keep clear of the subnormal range and overflow (the flag) only
    // beyond |phi| ~ 2^11.
    int e = 0;
    while ((1 << e) < N * N) ++e;
    const bool h = FMT == SPEC_F16;
    const float rho_store = h ? std::ldexp(1.0f, -e) : 1.0f, rho_load = h ? std::ldexp(1.0f, e) : 1.0f;
    const float phi_store = h ? 32.0f : 1.0f, phi_load = h ? 1.0f / 32.0f : 1.0f;
    if (ev) hipEventRecord(ev[0], s);
    const int nplanes = N * ntiles;
    const int blocks = std::min(nplanes, device_cus());
    if (PlaneSplit<N>::ok)
        hipLaunchKernelGGL((k_r2c_plane_w<N, FMT>), dim3(blocks), dim3(kPlaneThreads), 0, s, real_tiles, spec_tiles,
                           tw, nplanes, rho_store, flag);
    else
        hipLaunchKernelGGL((k_r2c_plane<N, FMT>), dim3(blocks), dim3(kPlaneThreads), 0, s, real_tiles, spec_tiles,
                           tw, nplanes, rho_store, flag);
    if (ev) hipEventRecord(ev[1], s);
    hipLaunchKernelGGL((k_zconv_half<N, FMT>), dim3(N * NH / 16, ntiles), dim3(kFftThreads), 0, s, spec_tiles, tw,
                       green, rho_load, phi_store, flag, lo, hi);
    if (ev) hipEventRecord(ev[2], s);
    const int out_planes = (hi - lo) * ntiles;
    if (PlaneSplit<N>::ok)
        hipLaunchKernelGGL((k_c2r_plane_w<N, FMT>), dim3(std::min(out_planes, device_cus())), dim3(kPlaneThreads),
                           0, s, spec_tiles, real_tiles, tw, out_planes, phi_load, lo, hi);
    else
        hipLaunchKernelGGL((k_c2r_plane<N, FMT>), dim3(std::min(out_planes, device_cus())), dim3(kPlaneThreads), 0,
                           s, spec_tiles, real_tiles, tw, out_planes, phi_load, lo, hi);
    if (ev) hipEventRecord(ev[3], s);
}

template <int N>
void launch_tiles(float* real_tiles, void* spec, int ntiles, const float2* tw, const float* green, int fmt,
                  int32_t* flag, int lo, int hi, hipStream_t s, hipEvent_t* ev) {
    if (fmt == SPEC_BF16) launch_tiles_fmt<N, SPEC_BF16>(real_tiles, spec, ntiles, tw, green, flag, lo, hi, s, ev);
    else if (fmt == SPEC_F16) launch_tiles_fmt<N, SPEC_F16>(real_tiles, spec, ntiles, tw, green, flag, lo, hi, s, ev);
    else launch_tiles_fmt<N, SPEC_F32>(real_tiles, spec, ntiles, tw, green, flag, lo, hi, s, ev);
}

using TilesFn = void (*)(float*, void*, int, const float2*, const float*, int, int32_t*, int, int, hipStream_t,
                         hipEvent_t*);

TilesFn tiles_for(int n) {
    switch (n) {
        case 32: return launch_tiles<32>;
        case 48: return launch_tiles<48>;
        case 64: return launch_tiles<64>;
        case 96: return launch_tiles<96>;
        case 128: return launch_tiles<128>;
        case 160: return launch_tiles<160>;
        case 192: return launch_tiles<192>;
        default: return nullptr;
    }
}

template <int N>
void launch_pass(float2* data, int batch, int kind, int mode, const float2* tw, const void* green,
                 hipStream_t s) {
    constexpr int W = pencils<N>();
    const unsigned blocks = (unsigned)((int64_t)N * N / W);
    dim3 grid(blocks, batch), block(kFftThreads);
#define CUBE_L(K, MO) hipLaunchKernelGGL((k_fft<N, K, MO>), grid, block, 0, s, data, tw, green)
    if (kind == 0) {
        if (mode == 0) CUBE_L(0, 0); else CUBE_L(0, 1);
    } else if (kind == 1) {
        if (mode == 0) CUBE_L(1, 0); else CUBE_L(1, 1);
    } else {
        if (mode == 0) CUBE_L(2, 0);
        else if (mode == 1) CUBE_L(2, 1);
        else if (mode == 2) CUBE_L(2, 2);
        else CUBE_L(2, 3);
    }
#undef CUBE_L
}

using PassFn = void (*)(float2*, int, int, int, const float2*, const void*, hipStream_t);

PassFn pass_for(int n) {
    switch (n) {
        case 16: return launch_pass<16>;
        case 32: return launch_pass<32>;
        case 48: return launch_pass<48>;
        case 64: return launch_pass<64>;
        case 80: return launch_pass<80>;
        case 96: return launch_pass<96>;
        case 112: return launch_pass<112>;
        case 128: return launch_pass<128>;
        case 160: return launch_pass<160>;
        case 192: return launch_pass<192>;
        case 224: return launch_pass<224>;
        case 256: return launch_pass<256>;
        case 320: return launch_pass<320>;
        case 384: return launch_pass<384>;
        case 448: return launch_pass<448>;
        case 512: return launch_pass<512>;
        case 1024: return launch_pass<1024>;
        default: return nullptr;
    }
}

}  // namespace

bool fft_supported(int n) { return pass_for(n) != nullptr; }

bool fft_tiles_supported(int n) { return tiles_for(n) != nullptr; }

void fft_tiles_convolve(float* real_tiles, void* spec_tiles, int n, int ntiles, const float2* tw,
                        const float* green_octant, int spec_format, int32_t* range_flag, int out_lo, int out_hi,
                        hipStream_t s, hipEvent_t* ev) {
    tiles_for(n)(real_tiles, spec_tiles, ntiles, tw, green_octant, spec_format, range_flag, out_lo, out_hi, s, ev);
}

void fft_make_twiddles(int n, float2* dev_table, hipStream_t s) {
    std::vector<float2> h(n);
    for (int k = 0; k < n; ++k) {
        // exact argument reduction: angle = 2 pi k / n in FP64, one rounding to FP32
        const double ang = 2.0 * M_PI * (double)k / (double)n;
        h[k] = make_float2((float)std::cos(ang), (float)(-std::sin(ang)));
    }
    hipMemcpyAsync(dev_table, h.data(), n * sizeof(float2), hipMemcpyHostToDevice, s);
    hipStreamSynchronize(s);
}

void fft3d(float2* data, int n, int batch, bool inverse, const float2* tw, hipStream_t s) {
    PassFn f = pass_for(n);
    const int mode = inverse ? 1 : 0;
    f(data, batch, 0, mode, tw, nullptr, s);
    f(data, batch, 1, mode, tw, nullptr, s);
    f(data, batch, 2, mode, tw, nullptr, s);
}

void fft3d_convolve(float2* data, int n, int batch, const float2* tw, const void* green_octant, int table_kind,
                    hipStream_t s, hipEvent_t* ev) {
    PassFn f = pass_for(n);
    if (ev) hipEventRecord(ev[0], s);
    f(data, batch, 0, 0, tw, nullptr, s);
    if (ev) hipEventRecord(ev[1], s);
    f(data, batch, 1, 0, tw, nullptr, s);
    if (ev) hipEventRecord(ev[2], s);
    f(data, batch, 2, table_kind == 0 ? 2 : 3, tw, green_octant, s);
    if (ev) hipEventRecord(ev[3], s);
    f(data, batch, 1, 1, tw, nullptr, s);
    if (ev) hipEventRecord(ev[4], s);
    f(data, batch, 0, 1, tw, nullptr, s);
    if (ev) hipEventRecord(ev[5], s);
}

}  // namespace cube
