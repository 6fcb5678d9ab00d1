// C ABI of libcube.so: context lifetime, device memory, and the order of the
// kernels in one particle-mesh step (Sec. II two-level PM on the compressed
// particles of Sec. III-A).
//
// Step order (every stage is a HIP kernel on the context stream):
//   prologue (velocity scale for the coming kick)
//   clear new counts
//   coarse deposit -> coarse FFT / x G_c / inverse FFT           (global mesh)
//   for each batch of tiles (fine meshes in flight):
//       fine deposit -> fine FFT / x G_f / inverse FFT -> gather+kick+drift+count
//   scan new counts -> new offsets
//   compaction (fast pull path, or the sorted general path)
//   epilogue (commit scale and max|u|), swap counts/offsets
// Particle buffers: A holds the state; the update writes B at the same index;
// compaction moves B back into A in the new order.
#include <algorithm>
#include <chrono>
#include <climits>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "ctx.h"

using namespace cube;

namespace {

thread_local std::string g_err;

}  // namespace

cube_status cube::fail(cube_status st, const std::string& msg) {
    g_err = msg;
    return st;
}

void cube::set_last_error(const char* msg) { g_err = msg ? msg : ""; }

namespace {

bool is_pow2(int v) { return v > 0 && (v & (v - 1)) == 0; }

// 32-point Gauss-Legendre rule on [-1, 1]: Newton's method on the Legendre
// polynomial from the usual cosine guesses.
struct GaussLegendre32 {
    double x[32], w[32];
    GaussLegendre32() {
        const int n = 32;
        for (int i = 0; i < n / 2; ++i) {
            double z = std::cos(M_PI * (i + 0.75) / (n + 0.5)), dp = 1.0;
            for (int it = 0; it < 100; ++it) {
                double p1 = 1.0, p0 = 0.0;
                for (int j = 1; j <= n; ++j) {
                    const double pm = p0;
                    p0 = p1;
                    p1 = ((2.0 * j - 1.0) * z * p0 - (j - 1.0) * pm) / j;
                }
                dp = n * (z * p1 - p0) / (z * z - 1.0);
                const double dz = p1 / dp;
                z -= dz;
                if (std::fabs(dz) < 1e-16) break;
            }
            x[i] = -z;
            x[n - 1 - i] = z;
            w[i] = w[n - 1 - i] = 2.0 / ((1.0 - z * z) * dp * dp);
        }
    }
};

// Expanding background: H(a) in units of H0, and the step's kick multiplier
// (3/2) Omega_m int da / (a^2 H) over [a - da/2, a + da/2] and drift
// multiplier int da / (a^3 H) over [a, a + da], rounded to FP32.
double hubble(double a, double om, double ol) { return std::sqrt(om / (a * a * a) + (1.0 - om - ol) / (a * a) + ol); }

void comoving_factors(const cube_box_desc& d, int64_t step, double* kick, float* drift) {
    static const GaussLegendre32 gl;
    const double om = d.omega_m, ol = d.omega_l, da = d.dt;
    const double a = (double)d.a_start + (double)step * da;
    auto integrate = [&](double a1, double a2, int power) {
        const double half = 0.5 * (a2 - a1), mid = 0.5 * (a2 + a1);
        double sum = 0.0;
        for (int i = 0; i < 32; ++i) {
            const double t = mid + half * gl.x[i];
            sum += gl.w[i] / (std::pow(t, power) * hubble(t, om, ol));
        }
        return half * sum;
    };
    *kick = 1.5 * om * integrate(a - 0.5 * da, a + 0.5 * da, 2);
    *drift = (float)integrate(a, a + da, 3);
}
int ilog2(int v) {
    int l = 0;
    while ((1 << l) < v) ++l;
    return l;
}

const char* const kStageNames[NSTAGES] = {
    "coarse_deposit", "coarse_fft_green", "fine_deposit", "fine_r2c_xy", "fine_z_green",
    "fine_c2r_xy", "gather_kick_drift", "scan_counts", "compact", "velocity_encode", "pp_force"};

}  // namespace

namespace {

}  // namespace


namespace {

cube_status validate(const cube_box_desc* d, Geom* out) {
    if (!d) return fail(CUBE_INVALID, "null descriptor");
    Geom g{};
    g.ns = d->n_side;
    g.f = d->fine_per_spacing;
    g.r = d->coarse_ratio;
    g.nt = d->tiles_per_dim;
    g.b = d->buffer_fine;
    g.a = d->r_cut_fine;
    if (g.ns <= 0 || g.nt <= 0 || g.a <= 0) return fail(CUBE_INVALID, "sizes must be positive");
    if (d->fd_order != 0 && d->fd_order != 2 && d->fd_order != 4)
        return fail(CUBE_INVALID, "fd_order must be 2 or 4 (0 means 2)");
    g.fdr = d->fd_order == 4 ? 2 : 1;
    if (d->vel_codec != CUBE_VEL_LINEAR && d->vel_codec != CUBE_VEL_CELL_MEAN)
        return fail(CUBE_INVALID, "unknown vel_codec");
    g.vcodec = d->vel_codec;
    // the pair search reaches one coarse cell each way (r_pp <= H)
    if (d->pp_range < 0 || d->pp_range > d->coarse_ratio || d->pp_range >= d->r_cut_fine)
        return fail(CUBE_INVALID, "pp_range must be in [0, coarse_ratio] and below r_cut_fine");
    g.npp = d->pp_range;
    if (d->comoving != 0 && d->comoving != 1) return fail(CUBE_INVALID, "comoving must be 0 or 1");
    if (d->comoving && !(d->omega_m > 0.0f && d->omega_l >= 0.0f && d->a_start > 0.0f &&
                         hubble(d->a_start, d->omega_m, d->omega_l) > 0.0))
        return fail(CUBE_INVALID, "comoving needs omega_m > 0, omega_l >= 0, a_start > 0 and H(a_start) > 0");
    if (!is_pow2(g.f) || !is_pow2(g.r) || g.r < 2 || g.r > 16 || g.r < g.f)
        return fail(CUBE_INVALID, "fine_per_spacing and coarse_ratio must be powers of two, 2 <= r <= 16, r >= f");
    const int64_t nfine = (int64_t)g.ns * g.f;
    if (nfine % g.r || nfine % g.nt) return fail(CUBE_INVALID, "n_side*f must be divisible by r and n_t");
    g.Nc = (int)(nfine / g.r);
    g.T = (int)(nfine / g.nt);
    if (g.T % g.r) return fail(CUBE_INVALID, "tile side must be a multiple of r");
    g.Tc = g.T / g.r;
    if (g.b % g.r) return fail(CUBE_INVALID, "buffer must be a multiple of r");
    if (g.nt == 1) {
        if (g.b != 0) return fail(CUBE_INVALID, "a single periodic tile has no buffer");
        if (2 * g.a >= g.T) return fail(CUBE_INVALID, "r_cut must be below half the box");
        g.F = g.T;
        g.periodic = 1;
    } else {
        // a target's CIC nodes lie within one cell of its tile, the gradient
        // reads fdr cells further, the truncated kernel a cells further, and
        // a density cell is complete one cell inside the buffer's edge
        if (g.a > g.b - 2 - g.fdr)
            return fail(CUBE_INVALID, g.fdr == 1 ? "tiles need r_cut <= buffer - 3"
                                                 : "tiles with 4-point gradients need r_cut <= buffer - 4");
        g.F = g.T + 2 * g.b;
        g.periodic = 0;
        if (g.F / g.r > g.Nc) return fail(CUBE_INVALID, "tile box larger than the periodic box");
    }
    g.Fc = g.F / g.r;
    g.hc = g.b / g.r;
    g.log2D = 9 - ilog2(g.r);
    g.ncells = (int64_t)g.Nc * g.Nc * g.Nc;
    g.n = (int64_t)g.ns * g.ns * g.ns;
    g.ntiles = g.nt * g.nt * g.nt;
    g.tc_shift = is_pow2(g.Tc) ? ilog2(g.Tc) : -1;
    g.nt_shift = is_pow2(g.nt) ? ilog2(g.nt) : -1;
    if (g.n >= (int64_t)1 << 31) return fail(CUBE_INVALID, "more than 2^31 - 1 particles");
    if (g.Nc % 4 || g.Nc < 10) return fail(CUBE_INVALID, "coarse mesh side must be a multiple of 4 and >= 12");
    if (!fft_supported(g.Nc) || !fft_tiles_supported(g.F))
        return fail(CUBE_UNSUPPORTED, "mesh side not supported by the FFT radix plans");
    if (!gather_supported(g))
        return fail(CUBE_UNSUPPORTED, "tile side must be a multiple of 32 fine cells and r in {4, 8}");
    if (!(d->dt > 0.0f) || !(d->v_headroom >= 1.0f)) return fail(CUBE_INVALID, "need dt > 0 and v_headroom >= 1");
    if (d->precision != CUBE_FP32 && d->precision != CUBE_MIXED_BF16 && d->precision != CUBE_MIXED_FP16)
        return fail(CUBE_INVALID, "unknown precision");
    *out = g;
    return CUBE_OK;
}

int batch_of(const Geom& g, const cube_box_desc& d) {
    const int b = d.tiles_per_batch > 0 ? d.tiles_per_batch : 64;
    return std::max(1, std::min(b, g.ntiles));
}

// per-block FP64 partial sums of the diagnostics (moments per chunk, potential per gather block)
int64_t partial_len(const Geom& g, int batch) {
    return std::max<int64_t>(4 * (g.ncells / g.Tc), (int64_t)gather_blocks_per_tile(g) * batch);
}

// Device bytes a context holds for its lifetime, and the largest set of
// temporaries any call adds on top (compress from host buffers, the general
// compaction path, the power spectrum, the Green's-table build).
struct Footprint {
    int64_t persistent;
    int64_t transient;
};

Footprint footprint_of(const Geom& g, const cube_box_desc& d) {
    const int batch = batch_of(g, d);
    const int64_t n = g.n, cells = g.ncells + 16;
    const int64_t Mc = g.Nc / 2 + 1, Mf = g.F / 2 + 1, F3 = (int64_t)g.F * g.F * g.F;
    int64_t p = 0;
    auto add = [&](int64_t bytes) { p += (int64_t)round256((size_t)bytes); };
    add(12 * n);
    if (d.with_ids) {
        add(4 * n);
        add(4 * n);
    }
    add(n);
    add(4 * n);
    add(16 * n);                                           // mover records
    add(4 * compact_bricks(g) * kHdrInts);                 // their brick headers
    add(4 * g.ntiles);                                     // per-tile record cursors
    for (int i = 0; i < 4; ++i) add(4 * cells);
    add(sizeof(StepScalars));
    add((int64_t)scan_workspace_bytes(cells));
    add(8 * g.ncells);
    add(8 * Mc * Mc * Mc);
    add(8 * (int64_t)g.Nc);
    add(4 * (batch * F3 + kFineRealPad));
    add(8 * (int64_t)batch * g.F * g.F * Mf);
    add(4 * Mf * Mf * Mf);
    add(8 * (int64_t)g.F);
    add(8 * 64);
    add(8 * partial_len(g, batch));
    if (g.vcodec) {
        add(24 * n);                   // FP32 working velocities, two sets of planes
        add(12 * g.ncells);            // cell means
        add(8 * 255);                  // tan table
    }
    if (g.npp) add(12 * n);            // PP accelerations
    auto r = [](int64_t bytes) { return (int64_t)round256((size_t)bytes); };
    const int64_t sortw = r((int64_t)sort_workspace_bytes(n));
    const int64_t t_green = r((int64_t)fine_green_workspace_bytes(g));
    const int64_t t_compress = 2 * r(12 * n) + 5 * r(4 * n) + r(256) + sortw;
    const int64_t t_general = 4 * r(4 * n) + sortw;
    const int64_t t_pk = r(8 * n) + r(8 * (int64_t)g.ns) + r(8 * 3 * (int64_t)g.ns * std::max(1, g.ns / 4 - 1));
    return {p, std::max(std::max(t_green, t_compress), std::max(t_general, t_pk))};
}

}  // namespace

namespace cube {

cube_status check_ctx(cube_ctx* c) {
    if (!c) return fail(CUBE_INVALID, "null context");
    if (c->poisoned) return fail(CUBE_DEVICE, "context poisoned by an earlier device error");
    return CUBE_OK;
}

cube_status launch_status(cube_ctx* c) {
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) {
        c->poisoned = true;
        return fail(CUBE_DEVICE, std::string("kernel launch: ") + hipGetErrorString(e));
    }
    return CUBE_OK;
}

cube_status sync(cube_ctx* c) {
    hipError_t e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) {
        c->poisoned = true;
        return fail(CUBE_DEVICE, std::string("stream: ") + hipGetErrorString(e));
    }
    return launch_status(c);
}

// coarse potential into ctx->coarse (real part)
void coarse_potential(cube_ctx* c) {
    const Geom& g = c->g;
    Profiler& P = c->prof;
    const double nc3 = (double)g.ncells;
    hipEvent_t e0 = P.on ? P.mark(c->stream) : nullptr;
    launch_coarse_deposit(g, c->offsets, c->A, c->coarse, nullptr, c->stream);
    hipEvent_t e1 = P.on ? P.mark(c->stream) : nullptr;
    fft3d_convolve(c->coarse, g.Nc, 1, c->tw_coarse, c->coarse_green, 1, c->stream);
    if (P.on) {
        hipEvent_t e2 = P.mark(c->stream);
        // deposit: complex mesh write + offsets read + 3 position bytes per particle
        P.add(ST_COARSE_DEP, e0, e1, 12.0 * nc3 + 3.0 * (double)g.n);
        // five read+write sweeps of the complex mesh
        P.add(ST_COARSE_FFT, e1, e2, 80.0 * nc3);
    }
}

StepPlan plan_of(const cube_ctx* c, bool force_fp32) {
    StepPlan p;
    p.wide = fine_deposit_needs_wide(c->g, c->max_block8);
    switch (c->desc.precision) {
        case CUBE_MIXED_BF16: p.fmt = 1; break;
        case CUBE_MIXED_FP16: p.fmt = (!force_fp32 && fp16_density_fits(c->g, c->max_block8)) ? 2 : 0; break;
        default: p.fmt = 0;
    }
    return p;
}

void fine_window(const Geom& g, bool full, int* lo, int* hi) {
    const bool whole = full || g.periodic;
    *lo = whole ? 0 : g.b - 1 - g.fdr;
    *hi = whole ? g.F : g.b + g.T + 1 + g.fdr;
}

// fine potentials of tiles [t0, t0 + nt) into ctx->fine_real: over the
// whole box when `full`, else over the tile plus the 1 + fdr cells the
// gather's interpolation and differences reach (all of the box for a
// periodic tile)
void fine_potential(cube_ctx* c, const StepPlan& plan, int t0, int nt, bool full = false) {
    const Geom& g = c->g;
    Profiler& P = c->prof;
    const int fmt = plan.fmt;
    int lo, hi;
    fine_window(g, full, &lo, &hi);
    hipEvent_t e0 = P.on ? P.mark(c->stream) : nullptr;
    launch_fine_deposit(g, c->offsets, c->A, t0, nt, c->fine_real, plan.wide, c->stream);
    if (!P.on) {
        fft_tiles_convolve(c->fine_real, c->fine_spec, g.F, nt, c->tw_fine, c->fine_green, fmt, &c->sc->overflow,
                           lo, hi, c->stream);
        return;
    }
    hipEvent_t ev[4];
    for (int i = 0; i < 4; ++i) ev[i] = P.get();
    fft_tiles_convolve(c->fine_real, c->fine_spec, g.F, nt, c->tw_fine, c->fine_green, fmt, &c->sc->overflow,
                       lo, hi, c->stream, ev);
    const double f3 = (double)g.F * g.F * g.F, fc3 = (double)g.Fc * g.Fc * g.Fc;
    // bytes per stored half-spectrum value: 8 (FP32) or 4 (16-bit pairs)
    const double h3 = (double)g.F * g.F * (g.F / 2 + 1) * (fmt == 0 ? 1.0 : 0.5);
    const double per_tile = (double)g.n / g.ntiles;
    const double src = per_tile * f3 / ((double)g.T * g.T * g.T);    // tile plus buffer
    // deposit: FP32 mesh write + offsets read + 3 position bytes per source
    P.add(ST_FINE_DEP, e0, ev[0], nt * (4.0 * f3 + 4.0 * fc3 + 3.0 * src));
    // xy planes: real mesh in, half spectrum out (and back); z: half spectrum in and out
    // z pass: every pencil in, only z in the window out; C2R: the window's
    // planes in, the window out
    const double wf = (double)(hi - lo) / g.F, w3 = (double)(hi - lo) * (hi - lo) * (hi - lo);
    P.add(ST_FFT_R2C, ev[0], ev[1], nt * (4.0 * f3 + 8.0 * h3));
    P.add(ST_FFT_ZG, ev[1], ev[2], nt * 8.0 * h3 * (1.0 + wf));
    P.add(ST_FFT_C2R, ev[2], ev[3], nt * (8.0 * h3 * wf + 4.0 * w3));
}

// extended PP accelerations of the current state (nothing when off)
void pp_forces(cube_ctx* c) {
    const Geom& g = c->g;
    if (!g.npp) return;
    Profiler& P = c->prof;
    hipEvent_t e0 = P.on ? P.mark(c->stream) : nullptr;
    launch_pp(g, c->offsets, c->A, c->pp, c->stream);
    // own positions and offsets, the neighbour cells' bytes (L2-resident), 12 B out
    if (P.on) P.add(ST_PP, e0, P.mark(c->stream), 15.0 * (double)g.n + 4.0 * (double)g.ncells);
}

GatherArgs gather_args(cube_ctx* c, int mode, int t0, int nt, int64_t step_index) {
    GatherArgs a{};
    a.g = c->g;
    a.offsets = c->offsets;
    a.in = c->A;
    a.out = c->B;
    a.dir = c->dir;
    a.far_key = c->far_key;
    a.ment = c->ment;
    a.mhdr = c->mhdr;
    a.tcursor = c->tcursor;
    a.counts_new = c->counts_new;
    a.fine_real = c->fine_real;
    a.coarse = c->coarse;
    a.sc = c->sc;
    a.vcell = c->vcell;
    for (int k = 0; k < 3; ++k) a.pp[k] = c->pp[k];
    a.kick = (double)c->desc.dt;
    a.drift = c->desc.dt;
    if (c->desc.comoving) comoving_factors(c->desc, step_index, &a.kick, &a.drift);
    a.tile0 = t0;
    a.ntiles = nt;
    a.mode = mode;
    return a;
}

void step_pre(cube_ctx* c) {
    const Geom& g = c->g;
    hipStream_t s = c->stream;
    StepScalars* sc = c->sc;
    launch_step_prologue(sc, c->desc.v_headroom, s);
    launch_fill_i32(c->counts_new, 0, g.ncells, s, &sc->halt);
    // the mover records of each tile go to the slots of its particles
    launch_strided_copy(c->offsets, (int64_t)g.Tc * g.Tc * g.Tc, c->tcursor, g.ntiles, s, &sc->halt);
    coarse_potential(c);
    pp_forces(c);
}

void step_gather(cube_ctx* c, int t0, int nt, const float* mesh, int64_t step_index) {
    const Geom& g = c->g;
    hipStream_t s = c->stream;
    Profiler& P = c->prof;
    GatherArgs a = gather_args(c, GATHER_STEP, t0, nt, step_index);
    a.fine_real = mesh;
    hipEvent_t e0 = P.on ? P.mark(s) : nullptr;
    launch_gather(a, s);
    if (P.on) {
        const double np = (double)g.n * nt / g.ntiles;
        const double t4 = (double)(g.T + 4) * (g.T + 4) * (g.T + 4);
        const double c4 = (double)(g.Tc + 4) * (g.Tc + 4) * (g.Tc + 4);
        // 6 B in, 7 B out (m', u', move code), one count update, potentials read once
        P.add(ST_GATHER, e0, P.mark(s), 21.0 * np + 4.0 * nt * (t4 + c4));
    }
}

void step_post(cube_ctx* c, const StepPlan& plan) {
    const Geom& g = c->g;
    hipStream_t s = c->stream;
    StepScalars* sc = c->sc;
    Profiler& P = c->prof;
    hipEvent_t es = P.on ? P.mark(s) : nullptr;
    launch_fill_i32(&sc->new_max_count, 0, 2, s, &sc->halt);     // new_max_count and new_max_block8
    exclusive_scan_i32(c->counts_new, c->offsets_new, g.ncells, c->scan_ws, s, &sc->new_max_count, &sc->halt);
    launch_max_block8(g, c->counts_new, &sc->new_max_block8, s, &sc->halt);
    if (P.on) P.add(ST_SCAN, es, P.mark(s), 8.0 * (double)g.ncells);
    if (c->dbg_force[2] > 0) {
        --c->dbg_force[2];
        launch_fill_i32(&sc->far_count, 1, 1, s, &sc->halt);
    }
    launch_step_decide(sc, INT_MAX, s);
    // with the cell-mean codec the kicked FP32 velocities move instead of codes
    Planes src = c->B, dst = c->A;
    if (g.vcodec)
        for (int k = 0; k < 3; ++k) src.u[k] = dst.u[k] = nullptr;
    hipEvent_t ec = P.on ? P.mark(s) : nullptr;
    launch_compact_bricks(g, c->offsets, c->offsets_new, c->dir, c->ment, c->mhdr, src, dst, sc, s);
    // 6 B + move code read, 6 B written, old and new offsets read
    if (P.on) P.add(ST_COMPACT, ec, P.mark(s), 13.0 * (double)g.n + 8.0 * (double)g.ncells);
    if (g.vcodec) {
        // re-encode against the new cells (sets sigma, max |u|, saturations)
        hipEvent_t ev = P.on ? P.mark(s) : nullptr;
        launch_vc_encode(g, c->offsets_new, c->A, c->vcell, sc, c->partial, s, true);
        // FP32 velocities read twice, codes written, cell means written
        if (P.on) P.add(ST_VENC, ev, P.mark(s), 27.0 * (double)g.n + 16.0 * (double)g.ncells);
    }
    launch_commit_cells(c->counts_new, c->offsets_new, c->counts, c->offsets, g.ncells, sc, s);
    launch_step_epilogue(sc, g, g.vcodec, plan.wide, plan.fmt == 2, s);
    if (c->dbg_force[3] > 0) {
        --c->dbg_force[3];
        launch_fill_i32(&sc->halt, 3, 1, s, &sc->halt);
    }
}

// Enqueue one step (no host synchronisation, no allocation): `plan` fixes
// the deposit width and spectrum format of this step and of the next one
// (checked by the epilogue), `step_index` the comoving factors.
void enqueue_step(cube_ctx* c, const StepPlan& plan, int64_t step_index) {
    const Geom& g = c->g;
    step_pre(c);
    for (int t0 = 0; t0 < g.ntiles; t0 += c->batch) {
        const int nt = std::min(c->batch, g.ntiles - t0);
        fine_potential(c, plan, t0, nt);
        if (t0 == 0 && c->dbg_force[1] > 0) {
            --c->dbg_force[1];
            launch_fill_i32(&c->sc->overflow, 1, 1, c->stream, &c->sc->halt);
        }
        step_gather(c, t0, nt, c->fine_real, step_index);
    }
    step_post(c, plan);
}

// Temporaries of the sorted general compaction: four key/index arrays of n
// words and the sort's workspace, from the context's allocator or from a
// caller-provided region.
size_t general_scratch_bytes(int64_t n) {
    return 4 * round256((size_t)n * sizeof(uint32_t)) + round256(sort_workspace_bytes(n));
}

// Finish a step that halted for the general compaction (halt 1): every
// stage up to the compaction has run and its outputs (the updated planes,
// move codes, far keys and new counts and offsets) are intact.  Sort the new
// keys stably, permute, re-encode (cell-mean codec), commit.  `scratch`
// (general_scratch_bytes) comes from the caller, or is allocated here.
cube_status finish_general(cube_ctx* c, const StepPlan& next, void* scratch) {
    const Geom& g = c->g;
    hipStream_t s = c->stream;
    launch_fill_i32(&c->sc->halt, 0, 1, s);
    Temp tmp(c->mem);
    char* base = static_cast<char*>(scratch);
    if (!base && !tmp.get(&base, general_scratch_bytes(g.n)))
        return fail(CUBE_OOM, "general compaction: out of memory");
    const size_t nb = round256((size_t)g.n * sizeof(uint32_t));
    uint32_t* key = reinterpret_cast<uint32_t*>(base);
    uint32_t* idx = reinterpret_cast<uint32_t*>(base + nb);
    uint32_t* kt = reinterpret_cast<uint32_t*>(base + 2 * nb);
    uint32_t* it = reinterpret_cast<uint32_t*>(base + 3 * nb);
    void* ws = base + 4 * nb;
    Planes src = c->B, dst = c->A;
    if (g.vcodec)
        for (int k = 0; k < 3; ++k) src.u[k] = dst.u[k] = nullptr;
    launch_general_keys(g, c->offsets, c->dir, c->far_key, key, idx, s);
    stable_sort_pairs(key, idx, kt, it, g.n, ilog2((int)std::min<int64_t>(g.ncells, 1 << 30)) + 1, ws, s);
    launch_permute_planes(idx, src, dst, g.n, s);
    if (g.vcodec) launch_vc_encode(g, c->offsets_new, c->A, c->vcell, c->sc, c->partial, s, true);
    launch_commit_cells(c->counts_new, c->offsets_new, c->counts, c->offsets, g.ncells, c->sc, s);
    launch_step_epilogue(c->sc, g, g.vcodec, next.wide, next.fmt == 2, s);
    return launch_status(c);
}

// Wait for the enqueued work and read the step scalars back.
cube_status read_scalars(cube_ctx* c) {
    CUBE_HIP(hipMemcpyAsync(c->sc_host, c->sc, sizeof(StepScalars), hipMemcpyDeviceToHost, c->stream));
    cube_status st = sync(c);
    if (st != CUBE_OK) return st;
    c->max_count = c->sc_host->max_count;
    c->max_block8 = c->sc_host->max_block8;
    return CUBE_OK;
}

cube_status resolve_halt(cube_ctx* c, void* scratch, bool* force_fp32, int64_t base_done) {
    const int halt = c->sc_host->halt;
    if (halt == 1) {
        cube_status st = finish_general(c, plan_of(c, *force_fp32), scratch);
        if (st == CUBE_OK) st = read_scalars(c);
        if (st != CUBE_OK) {
            launch_fill_i32(&c->sc->halt, 0, 1, c->stream);
            sync(c);
            return st;
        }
        if (c->sc_host->steps_done != base_done + 1) return fail(CUBE_DEVICE, "general compaction did not commit");
        c->step += 1;
        if (c->sc_host->halt == 3) launch_fill_i32(&c->sc->halt, 0, 1, c->stream);
    } else if (halt != 0) {
        // 2: FP16 overflow, the step is run again with FP32 spectra;
        // 3: the committed state needs another plan for the next step
        if (halt == 2) *force_fp32 = true;
        launch_fill_i32(&c->sc->halt, 0, 1, c->stream);
    }
    return CUBE_OK;
}

// nsteps steps: enqueue them all (one at a time after a recent halt), read
// the scalars once, resolve a halt, and continue with the rest.  scratch:
// optional region for the general compaction's temporaries.
cube_status run_steps(cube_ctx* c, int32_t nsteps, void* scratch) {
    int64_t done_total = 0;
    bool force_fp32 = false;
    bool met_halt = false;
    while (done_total < nsteps) {
        const StepPlan plan = plan_of(c, force_fp32);
        const int64_t k = c->halted_recently || met_halt ? 1 : nsteps - done_total;
        const int64_t base = c->sc_host->steps_done;
        for (int64_t i = 0; i < k; ++i) enqueue_step(c, plan, c->step + i);
        cube_status st = read_scalars(c);
        if (st != CUBE_OK) return st;
        if (c->prof.on) c->prof.flush();
        const int64_t done = c->sc_host->steps_done - base;
        c->step += done;
        done_total += done;
        if (c->sc_host->halt == 0) continue;
        met_halt = true;
        const int64_t before = c->step;
        st = resolve_halt(c, scratch, &force_fp32, base + done);
        if (st != CUBE_OK) return st;
        done_total += c->step - before;
    }
    c->halted_recently = met_halt;
    return CUBE_OK;
}

// Fixed device region for the callers that cannot allocate
// (cube_pm_step_noalloc): the temporaries of the sorted general compaction,
// 16 bytes per particle plus the sort's workspace, for boxes up to 128^3
// particles.  Each device holds its own copy for the life of the process;
// host code reaches it only through the address resolved per device below.
constexpr size_t kNoAllocScratchBytes = (size_t)36 << 20;

}  // namespace

static __device__ __align__(256) char scratch[kNoAllocScratchBytes];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};
bool g_scratch_tried[kMaxDevices] = {};

// Device address of `scratch` on the current device, resolved once per device
// with that device current (nullptr if the runtime refused).
void* noalloc_scratch_of_current_device() {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) {
        (void)hipGetLastError();
        return nullptr;
    }
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_tried[dev]) {
        g_scratch_tried[dev] = true;
        void* ptr = nullptr;
        if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) == hipSuccess) g_scratch_ptr[dev] = ptr;
        else (void)hipGetLastError();
    }
    return g_scratch_ptr[dev];
}

}  // namespace

extern "C" {

const char* cube_last_error(void) { return g_err.c_str(); }

cube_status cube_footprint(const cube_box_desc* desc, int64_t* persistent, int64_t* transient) {
    if (!persistent || !transient) return fail(CUBE_INVALID, "null output pointer");
    Geom g;
    cube_status st = validate(desc, &g);
    if (st != CUBE_OK) return st;
    const Footprint f = footprint_of(g, *desc);
    *persistent = f.persistent;
    *transient = f.transient;
    return CUBE_OK;
}

cube_status cube_init(const cube_box_desc* desc, const cube_allocator* alloc, void* hip_stream, cube_ctx** out) {
    if (!out) return fail(CUBE_INVALID, "null output pointer");
    *out = nullptr;
    if (alloc && (!alloc->alloc || !alloc->free)) return fail(CUBE_INVALID, "allocator needs alloc and free");
    Geom g;
    cube_status st = validate(desc, &g);
    if (st != CUBE_OK) return st;
    cube_ctx* c = new (std::nothrow) cube_ctx();
    if (!c) return fail(CUBE_OOM, "host allocation failed");
    c->g = g;
    c->desc = *desc;
    c->stream = static_cast<hipStream_t>(hip_stream);
    c->mem.stream = c->stream;
    if (alloc) {
        c->mem.custom = true;
        c->mem.al = *alloc;
    }
    const int64_t n = g.n;
    c->batch = batch_of(g, *desc);
    c->noalloc_scratch = noalloc_scratch_of_current_device();

#define CUBE_TRY(x)              \
    do {                         \
        cube_status s_ = (x);    \
        if (s_ != CUBE_OK) {     \
            delete c;            \
            return s_;           \
        }                        \
    } while (0)

    uint8_t* planes = nullptr;
    CUBE_TRY(c->alloc_n(&planes, 12 * n));
    for (int k = 0; k < 3; ++k) {
        c->A.m[k] = planes + k * n;
        c->A.u[k] = reinterpret_cast<int8_t*>(planes + (3 + k) * n);
        c->B.m[k] = planes + (6 + k) * n;
        c->B.u[k] = reinterpret_cast<int8_t*>(planes + (9 + k) * n);
    }
    if (desc->with_ids) {
        CUBE_TRY(c->alloc_n(&c->A.ids, n));
        CUBE_TRY(c->alloc_n(&c->B.ids, n));
    }
    if (g.npp) {
        float* pa = nullptr;
        CUBE_TRY(c->alloc_n(&pa, 3 * n));
        for (int k = 0; k < 3; ++k) c->pp[k] = pa + k * n;
    }
    double vtab_host[255];
    if (g.vcodec) {
        float* vp = nullptr;
        CUBE_TRY(c->alloc_n(&vp, 6 * n));
        float* vcp = nullptr;
        CUBE_TRY(c->alloc_n(&vcp, 3 * g.ncells));
        double* tab = nullptr;
        CUBE_TRY(c->alloc_n(&tab, 255));
        for (int k = 0; k < 3; ++k) {
            c->A.v[k] = vp + k * n;
            c->B.v[k] = vp + (3 + k) * n;
            c->vcell.vc[k] = vcp + k * g.ncells;
        }
        c->vcell.tab = tab;
        vc_table_host(vtab_host);
    }
    CUBE_TRY(c->alloc_n(&c->dir, n));
    CUBE_TRY(c->alloc_n(&c->far_key, n));
    CUBE_TRY(c->alloc_n(&c->ment, n));
    CUBE_TRY(c->alloc_n(&c->mhdr, compact_bricks(g) * kHdrInts));
    CUBE_TRY(c->alloc_n(&c->tcursor, g.ntiles));
    CUBE_TRY(c->alloc_n(&c->counts, g.ncells + 16));
    CUBE_TRY(c->alloc_n(&c->offsets, g.ncells + 16));
    CUBE_TRY(c->alloc_n(&c->counts_new, g.ncells + 16));
    CUBE_TRY(c->alloc_n(&c->offsets_new, g.ncells + 16));
    CUBE_TRY(c->alloc_n(&c->sc, 1));
    CUBE_TRY(c->alloc(&c->scan_ws, scan_workspace_bytes(g.ncells + 16)));
    CUBE_TRY(c->alloc_n(&c->coarse, g.ncells));
    const int64_t Mc = g.Nc / 2 + 1, Mf = g.F / 2 + 1;
    CUBE_TRY(c->alloc_n(&c->coarse_green, Mc * Mc * Mc));
    CUBE_TRY(c->alloc_n(&c->tw_coarse, g.Nc));
    const int64_t fcube = (int64_t)g.F * g.F * g.F;
    CUBE_TRY(c->alloc_n(&c->fine_real, (int64_t)c->batch * fcube + kFineRealPad));
    CUBE_TRY(c->alloc(&c->fine_spec, (size_t)c->batch * g.F * g.F * (g.F / 2 + 1) * sizeof(float2)));
    CUBE_TRY(c->alloc_n(&c->fine_green, Mf * Mf * Mf));
    CUBE_TRY(c->alloc_n(&c->tw_fine, g.F));
    CUBE_TRY(c->alloc_n(&c->reduced, 64));
    CUBE_TRY(c->alloc_n(&c->partial, partial_len(g, c->batch)));
    if (hipHostMalloc(reinterpret_cast<void**>(&c->sc_host), sizeof(StepScalars)) != hipSuccess) {
        c->sc_host = nullptr;
        delete c;
        return fail(CUBE_OOM, "pinned host allocation failed");
    }
    std::memset(c->sc_host, 0, sizeof(StepScalars));
    c->sc_host->s = 1.0;
    DevMem init_mem = c->mem;          // outlives c on the error paths below
    Temp init_tmp(init_mem);
    void* gws = nullptr;
    if (!init_tmp.get(&gws, fine_green_workspace_bytes(g))) {
        delete c;
        return fail(CUBE_OOM, "Green's table workspace");
    }

    // empty state, tables, twiddles
    hipStream_t s = c->stream;
    launch_fill_i32(c->counts, 0, g.ncells + 16, s);
    launch_fill_i32(c->offsets, 0, g.ncells + 16, s);
    if (hipMemcpyAsync(c->sc, c->sc_host, sizeof(StepScalars), hipMemcpyHostToDevice, s) != hipSuccess) {
        delete c;
        return fail(CUBE_DEVICE, "initial scalar copy failed");
    }
    if (g.vcodec) {
        launch_fill_i32(reinterpret_cast<int32_t*>(c->vcell.vc[0]), 0, 3 * g.ncells, s);   // zero means
        if (hipMemcpyAsync(const_cast<double*>(c->vcell.tab), vtab_host, sizeof(vtab_host), hipMemcpyHostToDevice,
                           s) != hipSuccess) {
            delete c;
            return fail(CUBE_DEVICE, "velocity table copy failed");
        }
    }
    build_coarse_green(g, c->coarse_green, s);
    build_fine_green(g, c->fine_green, gws, s);
    fft_make_twiddles(g.Nc, c->tw_coarse, s);
    fft_make_twiddles(g.F, c->tw_fine, s);
    if (hipStreamSynchronize(s) != hipSuccess || hipGetLastError() != hipSuccess) {
        delete c;
        return fail(CUBE_DEVICE, "initialisation kernels failed");
    }
#undef CUBE_TRY
    *out = c;
    return CUBE_OK;
}

void cube_destroy(cube_ctx* ctx) {
    if (!ctx) return;
    if (ctx->stream) hipStreamSynchronize(ctx->stream);
    delete ctx;
}

cube_status cube_compress(cube_ctx* c, const float* pos, const float* vel, int64_t n, int32_t on_device) {
    cube_status st = check_ctx(c);
    if (st != CUBE_OK) return st;
    const Geom& g = c->g;
    if (n != g.n || !pos || !vel) return fail(CUBE_INVALID, "compress needs n_side^3 particles");
    hipStream_t s = c->stream;
    Temp tmp(c->mem);
    const float* dpos = pos;
    const float* dvel = vel;
    float *hp = nullptr, *hv = nullptr;
    uint32_t *key = nullptr, *idx = nullptr, *kt = nullptr, *it = nullptr, *qp = nullptr, *vmax = nullptr;
    void* ws = nullptr;
    const size_t fb = (size_t)n * 3 * sizeof(float), ub = (size_t)n * sizeof(uint32_t);
    if (!on_device) {
        if (!tmp.get(&hp, fb) || !tmp.get(&hv, fb)) return fail(CUBE_OOM, "compress: staging allocation failed");
        if (hipMemcpyAsync(hp, pos, fb, hipMemcpyHostToDevice, s) != hipSuccess ||
            hipMemcpyAsync(hv, vel, fb, hipMemcpyHostToDevice, s) != hipSuccess) {
            c->poisoned = true;
            return fail(CUBE_DEVICE, "compress: upload failed");
        }
        dpos = hp;
        dvel = hv;
    }
    if (!tmp.get(&key, ub) || !tmp.get(&idx, ub) || !tmp.get(&kt, ub) || !tmp.get(&it, ub) || !tmp.get(&qp, ub) ||
        !tmp.get(&vmax, 256) || !tmp.get(&ws, sort_workspace_bytes(n)))
        return fail(CUBE_OOM, "compress: workspace allocation failed");
    launch_encode_keys(g, dpos, key, qp, idx, n, s);
    hipMemsetAsync(vmax, 0, sizeof(uint32_t), s);
    launch_absmax_f32(dvel, 3 * n, vmax, s);
    uint32_t vbits = 0;
    hipMemcpyAsync(&vbits, vmax, sizeof(uint32_t), hipMemcpyDeviceToHost, s);
    st = sync(c);
    if (st != CUBE_OK) return st;
    float vmaxf;
    std::memcpy(&vmaxf, &vbits, sizeof(float));
    double s0 = 1.0;
    if (vmaxf > 0.0f) {
        const double x = (double)c->desc.v_headroom * (double)vmaxf / 127.0;
        int e;
        const double m = std::frexp(x, &e);
        s0 = (m == 0.5) ? std::ldexp(1.0, e - 1) : std::ldexp(1.0, e);
    }
    int bits = ilog2((int)std::min<int64_t>(g.ncells, (int64_t)1 << 30));
    if (((int64_t)1 << bits) < g.ncells) ++bits;
    if (bits < 1) bits = 1;
    stable_sort_pairs(key, idx, kt, it, n, bits, ws, s);
    launch_fill_i32(c->counts, 0, g.ncells + 16, s);
    launch_count_keys(key, n, c->counts, s);
    StepScalars init{};
    init.s = s0;
    init.s_next = s0;
    *c->sc_host = init;
    hipMemcpyAsync(c->sc, c->sc_host, sizeof(StepScalars), hipMemcpyHostToDevice, s);
    exclusive_scan_i32(c->counts, c->offsets, g.ncells, c->scan_ws, s, &c->sc->max_count);
    launch_max_block8(g, c->counts, &c->sc->max_block8, s);
    launch_scatter_compressed(g, idx, qp, dvel, s0, c->A, c->counts, c->sc, n, s);
    if (g.vcodec) launch_vc_encode(g, c->offsets, c->A, c->vcell, c->sc, c->partial, s);
    hipMemcpyAsync(c->sc_host, c->sc, sizeof(StepScalars), hipMemcpyDeviceToHost, s);
    st = sync(c);
    if (st != CUBE_OK) return st;
    c->max_count = c->sc_host->max_count;
    c->max_block8 = c->sc_host->max_block8;
    c->has_state = true;
    c->step = 0;
    return CUBE_OK;
}

cube_status cube_decompress(cube_ctx* c, float* pos, float* vel, int64_t n, int32_t on_device) {
    cube_status st = check_ctx(c);
    if (st != CUBE_OK) return st;
    const Geom& g = c->g;
    if (n != g.n || !pos || !vel) return fail(CUBE_INVALID, "decompress needs n_side^3 particles");
    hipStream_t s = c->stream;
    float *dp = pos, *dv = vel;
    const size_t fb = (size_t)n * 3 * sizeof(float);
    Temp tmp(c->mem);
    if (!on_device && (!tmp.get(&dp, fb) || !tmp.get(&dv, fb))) return fail(CUBE_OOM, "decompress staging");
    launch_decode(g, c->offsets, c->A, c->sc, c->vcell, dp, dv, s);
    if (!on_device) {
        hipMemcpyAsync(pos, dp, fb, hipMemcpyDeviceToHost, s);
        hipMemcpyAsync(vel, dv, fb, hipMemcpyDeviceToHost, s);
    }
    return sync(c);
}

cube_status cube_pm_step(cube_ctx* c, int32_t nsteps) {
    cube_status st = check_ctx(c);
    if (st != CUBE_OK) return st;
    if (nsteps < 0) return fail(CUBE_INVALID, "negative step count");
    auto t0 = std::chrono::steady_clock::now();
    st = run_steps(c, nsteps, nullptr);
    auto t1 = std::chrono::steady_clock::now();
    if (st == CUBE_OK && nsteps > 0)
        c->last_step_ms = std::chrono::duration<double, std::milli>(t1 - t0).count() / nsteps;
    return st;
}

cube_status cube_pm_step_noalloc(cube_ctx* c, int32_t nsteps) {
    cube_status st = check_ctx(c);
    if (st != CUBE_OK) return st;
    if (nsteps < 0) return fail(CUBE_INVALID, "negative step count");
    if (general_scratch_bytes(c->g.n) > kNoAllocScratchBytes)
        return fail(CUBE_INVALID, "cube_pm_step_noalloc: the box needs " + std::to_string(general_scratch_bytes(c->g.n)) +
                                      " bytes of scratch, more than the fixed " +
                                      std::to_string(kNoAllocScratchBytes) + " (boxes up to 128^3 particles)");
    if (c->prof.on) return fail(CUBE_INVALID, "cube_pm_step_noalloc: profiling creates events; disable it");
    if (!c->noalloc_scratch) return fail(CUBE_DEVICE, "cube_pm_step_noalloc: scratch address not resolved");
    auto t0 = std::chrono::steady_clock::now();
    st = run_steps(c, nsteps, c->noalloc_scratch);
    auto t1 = std::chrono::steady_clock::now();
    if (st == CUBE_OK && nsteps > 0)
        c->last_step_ms = std::chrono::duration<double, std::milli>(t1 - t0).count() / nsteps;
    return st;
}

cube_status cube_forces(cube_ctx* c, float* acc, int32_t on_device) {
    cube_status st = check_ctx(c);
    if (st != CUBE_OK) return st;
    if (!acc) return fail(CUBE_INVALID, "null output");
    const Geom& g = c->g;
    hipStream_t s = c->stream;
    float* dacc = acc;
    const size_t bytes = (size_t)g.n * 3 * sizeof(float);
    Temp tmp(c->mem);
    if (!on_device && !tmp.get(&dacc, bytes)) return fail(CUBE_OOM, "forces staging");
    // a FP16 potential spectrum out of range: evaluate again with FP32 spectra
    for (int attempt = 0; attempt < 2; ++attempt) {
        const StepPlan plan = plan_of(c, attempt > 0);
        launch_fill_i32(&c->sc->overflow, 0, 1, s);
        coarse_potential(c);
        pp_forces(c);
        for (int t0 = 0; t0 < g.ntiles; t0 += c->batch) {
            const int nt = std::min(c->batch, g.ntiles - t0);
            fine_potential(c, plan, t0, nt);
            GatherArgs a = gather_args(c, GATHER_FORCE, t0, nt, c->step);
            a.acc = dacc;
            launch_gather(a, s);
        }
        int32_t oflow = 0;
        CUBE_HIP(hipMemcpyAsync(&oflow, &c->sc->overflow, sizeof(int32_t), hipMemcpyDeviceToHost, s));
        st = sync(c);
        if (st != CUBE_OK) return st;
        if (!oflow) break;
        if (attempt > 0) return fail(CUBE_OVERFLOW, "FP32 spectra raised the FP16 range flag");
    }
    if (!on_device) {
        CUBE_HIP(hipMemcpyAsync(acc, dacc, bytes, hipMemcpyDeviceToHost, s));
        st = sync(c);
    }
    return st;
}

cube_status cube_get_state(cube_ctx* c, cube_state_view* v) {
    cube_status st = check_ctx(c);
    if (st != CUBE_OK) return st;
    const Geom& g = c->g;
    if (!v || v->n_particles != g.n || v->n_cells != g.ncells) return fail(CUBE_INVALID, "state view size mismatch");
    hipStream_t s = c->stream;
    const hipMemcpyKind kind = v->on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
    for (int k = 0; k < 3; ++k) {
        if (v->m[k]) CUBE_HIP(hipMemcpyAsync(v->m[k], c->A.m[k], g.n, kind, s));
        if (v->u[k]) CUBE_HIP(hipMemcpyAsync(v->u[k], c->A.u[k], g.n, kind, s));
    }
    if (v->counts) CUBE_HIP(hipMemcpyAsync(v->counts, c->counts, g.ncells * sizeof(int32_t), kind, s));
    if (v->ids && c->A.ids) CUBE_HIP(hipMemcpyAsync(v->ids, c->A.ids, g.n * sizeof(uint32_t), kind, s));
    if (g.vcodec)
        for (int k = 0; k < 3; ++k)
            if (v->vc[k]) CUBE_HIP(hipMemcpyAsync(v->vc[k], c->vcell.vc[k], g.ncells * sizeof(float), kind, s));
    CUBE_HIP(hipMemcpyAsync(c->sc_host, c->sc, sizeof(StepScalars), hipMemcpyDeviceToHost, s));
    st = sync(c);
    if (st != CUBE_OK) return st;
    v->s_v = c->sc_host->s;
    v->max_u = c->sc_host->max_u;
    v->step = c->step;
    return CUBE_OK;
}

cube_status cube_set_state(cube_ctx* c, const cube_state_view* v) {
    cube_status st = check_ctx(c);
    if (st != CUBE_OK) return st;
    const Geom& g = c->g;
    if (!v || v->n_particles != g.n || v->n_cells != g.ncells || !v->counts)
        return fail(CUBE_INVALID, "state view size mismatch");
    if (!(v->s_v > 0.0) || v->max_u < 0 || v->max_u > 127) return fail(CUBE_INVALID, "bad velocity scale or max_u");
    for (int k = 0; k < 3; ++k) {
        if (!v->m[k] || !v->u[k]) return fail(CUBE_INVALID, "missing planes");
        if (g.vcodec && !v->vc[k]) return fail(CUBE_INVALID, "the cell-mean codec needs the cell means vc");
    }
    hipStream_t s = c->stream;
    const hipMemcpyKind kind = v->on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
    for (int k = 0; k < 3; ++k) {
        CUBE_HIP(hipMemcpyAsync(c->A.m[k], v->m[k], g.n, kind, s));
        CUBE_HIP(hipMemcpyAsync(c->A.u[k], v->u[k], g.n, kind, s));
    }
    CUBE_HIP(hipMemcpyAsync(c->counts, v->counts, g.ncells * sizeof(int32_t), kind, s));
    if (g.vcodec)
        for (int k = 0; k < 3; ++k)
            CUBE_HIP(hipMemcpyAsync(c->vcell.vc[k], v->vc[k], g.ncells * sizeof(float), kind, s));
    if (c->A.ids) {
        if (v->ids) CUBE_HIP(hipMemcpyAsync(c->A.ids, v->ids, g.n * sizeof(uint32_t), kind, s));
        else CUBE_HIP(hipMemsetAsync(c->A.ids, 0, g.n * sizeof(uint32_t), s));
    }
    StepScalars init{};
    init.s = v->s_v;
    init.s_next = v->s_v;
    init.max_u = v->max_u;
    *c->sc_host = init;
    CUBE_HIP(hipMemcpyAsync(c->sc, c->sc_host, sizeof(StepScalars), hipMemcpyHostToDevice, s));
    // the counts must be non-negative and sum to n (in 64 bits) before any
    // offset derived from them indexes the particle planes
    long long check[2] = {0, INT64_MAX};
    long long* dcheck = reinterpret_cast<long long*>(c->reduced);
    CUBE_HIP(hipMemcpyAsync(dcheck, check, sizeof(check), hipMemcpyHostToDevice, s));
    launch_count_check(c->counts, g.ncells, dcheck, s);
    CUBE_HIP(hipMemcpyAsync(check, dcheck, sizeof(check), hipMemcpyDeviceToHost, s));
    st = sync(c);
    if (st != CUBE_OK) return st;
    if (check[1] < 0 || check[0] != (long long)g.n) {
        // never leave offsets that point past the particle arrays
        launch_fill_i32(c->counts, 0, g.ncells + 16, s);
        launch_fill_i32(c->offsets, 0, g.ncells + 16, s);
        c->has_state = false;
        sync(c);
        return fail(CUBE_INVALID, check[1] < 0 ? "negative cell count" : "counts do not sum to n_particles");
    }
    exclusive_scan_i32(c->counts, c->offsets, g.ncells, c->scan_ws, s, &c->sc->max_count);
    launch_max_block8(g, c->counts, &c->sc->max_block8, s);
    CUBE_HIP(hipMemcpyAsync(c->sc_host, c->sc, sizeof(StepScalars), hipMemcpyDeviceToHost, s));
    st = sync(c);
    if (st != CUBE_OK) return st;
    c->max_count = c->sc_host->max_count;
    c->max_block8 = c->sc_host->max_block8;
    c->has_state = true;
    c->step = v->step;
    return CUBE_OK;
}

cube_status cube_diagnostics(cube_ctx* c, cube_diag* out) {
    cube_status st = check_ctx(c);
    if (st != CUBE_OK) return st;
    if (!out) return fail(CUBE_INVALID, "null output");
    const Geom& g = c->g;
    hipStream_t s = c->stream;
    const int chunks = (int)(g.ncells / g.Tc);
    std::memset(out, 0, sizeof(*out));
    launch_moments(g, c->offsets, c->A, c->sc, c->vcell, c->partial, chunks, s);
    launch_reduce_partials(c->partial, chunks, 4, c->reduced, s);
    double mom[4];
    CUBE_HIP(hipMemcpyAsync(mom, c->reduced, sizeof(mom), hipMemcpyDeviceToHost, s));
    int32_t total = 0;
    CUBE_HIP(hipMemcpyAsync(&total, c->offsets + g.ncells, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    CUBE_HIP(hipMemcpyAsync(c->sc_host, c->sc, sizeof(StepScalars), hipMemcpyDeviceToHost, s));
    st = sync(c);
    if (st != CUBE_OK) return st;
    out->mass = total;
    out->momentum[0] = mom[0];
    out->momentum[1] = mom[1];
    out->momentum[2] = mom[2];
    out->kinetic = 0.5 * mom[3];
    out->saturations = c->sc_host->saturations;
    out->max_carry = c->sc_host->max_carry;
    out->max_u = c->sc_host->max_u;
    out->s_v = c->sc_host->s;
    out->step = c->step;
    out->last_step_ms = c->last_step_ms;
    // potential energy: 1/2 sum over particles of phi_f + phi_c at their
    // positions (again with FP32 spectra if a FP16 one left its range)
    double wsum = 0.0;
    std::vector<double> part;
    for (int attempt = 0; attempt < 2; ++attempt) {
        const StepPlan plan = plan_of(c, attempt > 0);
        launch_fill_i32(&c->sc->overflow, 0, 1, s);
        coarse_potential(c);
        wsum = 0.0;
        for (int t0 = 0; t0 < g.ntiles; t0 += c->batch) {
            const int nt = std::min(c->batch, g.ntiles - t0);
            fine_potential(c, plan, t0, nt);
            GatherArgs a = gather_args(c, GATHER_POTENTIAL, t0, nt, c->step);
            a.partial = c->partial;
            launch_gather(a, s);
            const int64_t np = (int64_t)gather_blocks_per_tile(g) * nt;
            part.resize(np);
            CUBE_HIP(hipMemcpyAsync(part.data(), c->partial, np * sizeof(double), hipMemcpyDeviceToHost, s));
            st = sync(c);
            if (st != CUBE_OK) return st;
            for (double v : part) wsum += v;
        }
        int32_t oflow = 0;
        CUBE_HIP(hipMemcpyAsync(&oflow, &c->sc->overflow, sizeof(int32_t), hipMemcpyDeviceToHost, s));
        st = sync(c);
        if (st != CUBE_OK) return st;
        if (!oflow) break;
        if (attempt > 0) return fail(CUBE_OVERFLOW, "FP32 spectra raised the FP16 range flag");
    }
    out->potential = 0.5 * wsum;
    return CUBE_OK;
}

cube_status cube_power_spectrum(cube_ctx* c, int32_t nbins, double* k, double* pk, int64_t* nmodes) {
    cube_status st = check_ctx(c);
    if (st != CUBE_OK) return st;
    const Geom& g = c->g;
    const int n = g.ns;
    if (nbins != n / 4 - 1 || !k || !pk || !nmodes) return fail(CUBE_INVALID, "nbins must be n_side/4 - 1");
    if (!fft_supported(n) || g.r < g.f) return fail(CUBE_UNSUPPORTED, "diagnostic mesh size not supported");
    hipStream_t s = c->stream;
    float2* mesh = nullptr;
    float2* tw = nullptr;
    double* part = nullptr;
    const int64_t cells = (int64_t)n * n * n;
    Temp tmp(c->mem);
    if (!tmp.get(&mesh, cells * sizeof(float2)) || !tmp.get(&tw, n * sizeof(float2)) ||
        !tmp.get(&part, (size_t)n * 3 * nbins * sizeof(double)))
        return fail(CUBE_OOM, "P(k) workspace");
    fft_make_twiddles(n, tw, s);
    launch_diag_deposit(g, c->offsets, c->A, mesh, s);
    fft3d(mesh, n, 1, false, tw, s);
    launch_power_bins(mesh, n, nbins, part, n, s);
    std::vector<double> h((size_t)n * 3 * nbins);
    hipMemcpyAsync(h.data(), part, h.size() * sizeof(double), hipMemcpyDeviceToHost, s);
    st = sync(c);
    if (st != CUBE_OK) return st;
    for (int j = 0; j < nbins; ++j) {
        double ps = 0.0, ks = 0.0, cs = 0.0;
        for (int z = 0; z < n; ++z) {
            ps += h[(size_t)z * 3 * nbins + j];
            ks += h[(size_t)z * 3 * nbins + nbins + j];
            cs += h[(size_t)z * 3 * nbins + 2 * nbins + j];
        }
        nmodes[j] = (int64_t)llround(cs);
        pk[j] = cs > 0 ? ps / cs : 0.0;
        k[j] = cs > 0 ? ks / cs : 0.0;
    }
    return CUBE_OK;
}

cube_status cube_debug_mesh(cube_ctx* c, int32_t what, int32_t tile, float* out) {
    cube_status st = check_ctx(c);
    if (st != CUBE_OK) return st;
    const Geom& g = c->g;
    if (!out) return fail(CUBE_INVALID, "null output");
    hipStream_t s = c->stream;
    if (what == 0 || what == 1) {
        if (what == 0) launch_coarse_deposit(g, c->offsets, c->A, c->coarse, nullptr, s);
        else coarse_potential(c);
        CUBE_HIP(hipMemcpy2DAsync(out, sizeof(float), c->coarse, sizeof(float2), sizeof(float), g.ncells,
                                  hipMemcpyDeviceToDevice, s));
    } else if (what == 2 || what == 3) {
        if (tile < 0 || tile >= g.ntiles) return fail(CUBE_INVALID, "tile out of range");
        const int64_t fcube = (int64_t)g.F * g.F * g.F;
        if (what == 2)
            launch_fine_deposit(g, c->offsets, c->A, tile, 1, c->fine_real, fine_deposit_needs_wide(g, c->max_block8),
                                s);
        else fine_potential(c, plan_of(c), tile, 1, true);
        CUBE_HIP(hipMemcpyAsync(out, c->fine_real, fcube * sizeof(float), hipMemcpyDeviceToDevice, s));
    } else {
        return fail(CUBE_INVALID, "unknown mesh");
    }
    return sync(c);
}

cube_status cube_debug_force(cube_ctx* c, int32_t what, int32_t count) {
    cube_status st = check_ctx(c);
    if (st != CUBE_OK) return st;
    if (what < 1 || what > 3 || count < 0) return fail(CUBE_INVALID, "unknown forced condition");
    c->dbg_force[what] = count;
    return CUBE_OK;
}

cube_status cube_fft3d(int32_t n, float* data, int32_t inverse, void* hip_stream) {
    if (!data) return fail(CUBE_INVALID, "null data");
    if (!fft_supported(n)) return fail(CUBE_UNSUPPORTED, "size not supported by the radix plans");
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    float2* tw = nullptr;
    CUBE_HIP(hipMalloc(&tw, n * sizeof(float2)));
    fft_make_twiddles(n, tw, s);
    fft3d(reinterpret_cast<float2*>(data), n, 1, inverse != 0, tw, s);
    hipError_t e = hipStreamSynchronize(s);
    hipFree(tw);
    if (e != hipSuccess) return fail(CUBE_DEVICE, hipGetErrorString(e));
    e = hipGetLastError();
    if (e != hipSuccess) return fail(CUBE_DEVICE, hipGetErrorString(e));
    return CUBE_OK;
}

cube_status cube_profile_enable(cube_ctx* c, int32_t enable) {
    cube_status st = check_ctx(c);
    if (st != CUBE_OK) return st;
    st = sync(c);
    if (st != CUBE_OK) return st;
    c->prof.flush();
    c->prof.reset();
    c->prof.on = enable != 0;
    return CUBE_OK;
}

cube_status cube_profile_read(cube_ctx* c, cube_stage_stat* out, int32_t max, int32_t* n) {
    cube_status st = check_ctx(c);
    if (st != CUBE_OK) return st;
    if (!out || !n || max < 0) return fail(CUBE_INVALID, "bad profile buffer");
    st = sync(c);
    if (st != CUBE_OK) return st;
    c->prof.flush();
    int k = 0;
    for (int i = 0; i < NSTAGES && k < max; ++i) {
        std::memset(&out[k], 0, sizeof(cube_stage_stat));
        std::snprintf(out[k].name, sizeof(out[k].name), "%s", kStageNames[i]);
        out[k].launches = c->prof.launches[i];
        out[k].total_ms = c->prof.ms[i];
        out[k].bytes = c->prof.bytes[i];
        ++k;
    }
    *n = k;
    return CUBE_OK;
}

}  // extern "C"
