/*
 * cube.h -- C ABI of libcube.so, an MI355X (gfx950) implementation of the
 * per-step force-and-update loop of CUBE's two-level particle-mesh (PMPM)
 * method on fixed-point-compressed particles (Cheng et al., arXiv:2003.03931).
 *
 * What one step computes (Sec. II and Sec. III-A of the paper):
 *   decode the 1-byte cell-relative position offsets (Eq. (2)) of particles
 *   stored cell-ordered with a per-cell count; deposit mass by cloud-in-cell
 *   onto one global periodic coarse mesh and onto the fine mesh of every tile
 *   (tile plus buffer); solve Poisson on each mesh by FFT, Green's-function
 *   multiply and inverse FFT (Eq. (1) with the force-split kernels);
 *   difference the potentials, interpolate the force back to the particles,
 *   kick and requantise the 1-byte velocities, drift and requantise the
 *   1-byte positions, then recount and stably compact the particles by cell.
 *
 * Conventions where the paper is silent (units, codec details, Green's
 * functions, integrator, order), in brief:
 * lengths in mean inter-particle spacings, particle mass 1, lap(phi) = rho - 1,
 * positions x = (256 n_c + m + 1/2) H / 256 (0-based n_c, H the coarse cell
 * size), velocities v = u * s with int8 u and a power-of-two scale s per box,
 * kick-drift leapfrog, canonical cell order tile-major then x-fastest.
 *
 * Every entry point returns a cube_status (0 == CUBE_OK); no C++ exception
 * crosses this boundary.  cube_last_error() returns a thread-local message
 * describing the last failure on the calling thread.  All device work is
 * enqueued on the stream given to cube_init.  A context is used by one host
 * thread at a time.
 */
#ifndef CUBE_H
#define CUBE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    CUBE_OK = 0,
    CUBE_INVALID = 1,      /* bad descriptor, geometry or argument; ctx unchanged     */
    CUBE_OOM = 2,          /* device allocation failed; ctx unchanged                 */
    CUBE_DEVICE = 3,       /* HIP runtime error; ctx is poisoned (only destroy valid) */
    CUBE_NOT_READY = 4,    /* cube_poll: the request is queued or running             */
    CUBE_OVERFLOW = 5,     /* FP32 spectra still raised the FP16 range flag (not seen) */
    CUBE_UNSUPPORTED = 6   /* mesh side not factorable by the FFT radices             */
} cube_status;

/*
 * Precision of the fine-mesh work.  Deposits are exact fixed point in every
 * mode, and every FFT pass, Green's multiply, gradient, interpolation and kick
 * computes in FP32.  The modes differ only in how the half spectra of the tile
 * meshes are stored in HBM between the three FFT sweeps (the largest traffic
 * of the step):
 *   CUBE_FP32        FP32 complex (8 bytes per value).
 *   CUBE_MIXED_BF16  BF16 real and imaginary parts (4 bytes), rounded to
 *                    nearest even; about 2^-9 relative error per stored value.
 *   CUBE_MIXED_FP16  FP16 parts scaled by a power of two (4 bytes); about
 *                    2^-12 relative error per value.  Steps whose densities
 *                    could leave the FP16 range are run with FP32 storage,
 *                    and so is again any step in which a potential spectrum
 *                    value left it.
 */
typedef enum {
    CUBE_FP32 = 0,
    CUBE_MIXED_BF16 = 1,
    CUBE_MIXED_FP16 = 2
} cube_precision;

/*
 * Velocity storage (Sec. III-A), one signed byte u per axis and particle in
 * both cases:
 *   CUBE_VEL_LINEAR     v = u s with one power-of-two scale s per box.
 *   CUBE_VEL_CELL_MEAN  Eq. (3): v = v_c + sigma tan(u pi / 255), v_c the FP32
 *                       mean velocity of the particle's coarse cell (three
 *                       floats per cell, summed sequentially in storage
 *                       order), sigma the power of two at or above the rms
 *                       deviation; codes are encoded with the fast arctangent
 *                       of Eq. (4).  In a step the kicked velocity is held in
 *                       FP32 (24 bytes per particle of working planes) and
 *                       re-encoded against the new cells after the
 *                       reordering.
 */
typedef enum {
    CUBE_VEL_LINEAR = 0,
    CUBE_VEL_CELL_MEAN = 1
} cube_vel_codec;

/*
 * Box geometry (Sec. II: coarse mesh, tiles with buffers; Sec. III-A: the
 * coarse mesh also defines the position codec).
 *   n_side            particles per dimension; box side L = n_side spacings.
 *   tiles_per_dim     n_t; the fine meshes are per tile.  1 = one periodic tile.
 *   fine_per_spacing  f, fine cells per spacing (power of two).
 *   coarse_ratio      r, fine cells per coarse cell (power of two, 2..16).
 *   buffer_fine       b, tile buffer in fine cells (multiple of r; 0 if n_t == 1).
 *   r_cut_fine        a, force-split radius in fine cells; needs a <= b - 3
 *                     (n_t > 1, 2-point gradients), a <= b - 4 (n_t > 1,
 *                     4-point gradients) or 2a < tile side (n_t == 1).
 *   dt                time step (units of the dynamical time).
 *   v_headroom        h_v >= 1, velocity-scale headroom (2 is the default).
 *   precision         cube_precision.
 *   with_ids          nonzero: carry a uint32 particle id plane (tests only; not
 *                     part of the 6 bytes per particle).
 *   tiles_per_batch   tiles whose fine meshes are in flight at once (0 = auto).
 *   fd_order          central-difference gradient of both potentials (Sec. II,
 *                     Eq. (1) taken through the potential): 2 = two-point
 *                     (phi(c+1) - phi(c-1)) / 2h, 4 = four-point
 *                     (8 (phi(c+1) - phi(c-1)) - (phi(c+2) - phi(c-2))) / 12h;
 *                     0 means 2, anything else is CUBE_INVALID.
 *   vel_codec         cube_vel_codec (0 = linear bytes, the default).
 *   comoving          0: static background, dt is the time step.  1: expanding
 *                     background (the paper's LambdaCDM setting, Sec. IV):
 *                     positions comoving, velocities the canonical momentum
 *                     p = a^2 dx/dt (time in 1/H0), dt the step in the scale
 *                     factor a, step n at a = a_start + n dt.  A step kicks by
 *                     the force times (3/2) omega_m int da / (a^2 H) over
 *                     [a - dt/2, a + dt/2] and drifts by p times
 *                     int da / (a^3 H) over [a, a + dt] (rounded to FP32),
 *                     H = sqrt(omega_m a^-3 + (1 - omega_m - omega_l) a^-2 + omega_l).
 *   omega_m, omega_l  density parameters (comoving only; omega_m > 0).
 *   a_start           scale factor of the state at step 0 (comoving only; > 0).
 *   pp_range          extended PP force (Sec. II, optional module): 0 = off;
 *                     n_pp in [1, coarse_ratio] and below r_cut_fine: pairs
 *                     closer than r_pp = n_pp fine cells attract explicitly by
 *                     F_G(r) - F_S2(r; r_pp) (F_S2 the attraction of two S2
 *                     clouds of diameter r_pp, equal to F_G from r_pp on, so
 *                     the pair force vanishes there), and the fine kernel
 *                     leaves that part out:
 *                     -(S_pp^2 - S^2) / k^2.  Pair distances come from the
 *                     integer positions (exact squared separations in
 *                     position quanta).  Costs 12 bytes per particle of
 *                     device memory.  Anything else is CUBE_INVALID.
 * Derived: coarse cells per side N_c = n_side f / r, tile side T = n_side f / n_t
 * fine cells, tile FFT box F = T + 2b; every FFT side must factor into 2,3,5,7.
 */
typedef struct {
    int32_t n_side;
    int32_t tiles_per_dim;
    int32_t fine_per_spacing;
    int32_t coarse_ratio;
    int32_t buffer_fine;
    int32_t r_cut_fine;
    float dt;
    float v_headroom;
    int32_t precision;
    int32_t with_ids;
    int32_t tiles_per_batch;
    int32_t fd_order;
    int32_t vel_codec;
    int32_t comoving;
    float omega_m;
    float omega_l;
    float a_start;
    int32_t pp_range;
} cube_box_desc;

typedef struct cube_ctx cube_ctx;

/*
 * Caller-owned buffers describing a compressed state (Sec. III-A: six 1-byte
 * integers per particle plus the per-cell counts).  Used by cube_get_state
 * (library copies out) and cube_set_state (library copies in).
 *   m[3]      uint8 position offsets per axis, n_particles each, canonical order.
 *   u[3]      int8 velocity codes per axis, n_particles each.
 *   counts    int32 particle count per coarse cell, N_c^3 entries, canonical
 *             cell order (tile-major, tile index x-fastest; x-fastest inside).
 *   ids       uint32 ids (only with with_ids; may be NULL otherwise).
 *   s_v       velocity scale (a power of two; sigma with CUBE_VEL_CELL_MEAN),
 *             M_u = max |u| of the stored u, step = number of steps taken.
 *   on_device nonzero: the pointers are device pointers, else host pointers.
 *   vc[3]     CUBE_VEL_CELL_MEAN only: FP32 cell-mean velocity per axis, N_c^3
 *             entries each in canonical cell order (required by set_state,
 *             filled by get_state when non-NULL; ignored otherwise).
 */
typedef struct {
    int64_t n_particles;
    int64_t n_cells;
    uint8_t* m[3];
    int8_t* u[3];
    int32_t* counts;
    uint32_t* ids;
    double s_v;
    int32_t max_u;
    int32_t on_device;
    int64_t step;
    float* vc[3];
} cube_state_view;

/* FP64 diagnostics of the current state (mass and momentum sums, energies)
 * plus counters accumulated by cube_pm_step. */
typedef struct {
    int64_t mass;              /* sum of counts (exact)                              */
    double momentum[3];        /* sum of decoded velocities, FP64                    */
    double kinetic;            /* 1/2 sum v^2, FP64                                  */
    double potential;          /* 1/2 sum phi(x_i), FP64 sum of FP32 potentials      */
    int64_t saturations;       /* velocity components clamped to +-127 so far        */
    int32_t max_carry;         /* largest |cell carry| of the last step              */
    int32_t max_u;             /* max |u| of the state                               */
    double s_v;                /* velocity scale of the state                        */
    int64_t step;              /* steps taken                                        */
    double last_step_ms;       /* host wall time of the last cube_pm_step call / step */
} cube_diag;

/* Thread-local description of the last failure (empty if none). */
const char* cube_last_error(void);

/*
 * Device memory callbacks.  The library obtains every device buffer it uses
 * (state, meshes, tables, workspace, and the temporaries of single calls)
 * through them.  alloc returns at least `bytes` bytes of device memory usable
 * in stream order on hip_stream, or NULL on failure (the call then returns
 * CUBE_OOM); free receives the pointer with the same `bytes`.  Temporaries are
 * freed right after the stream work that used them was enqueued, so a
 * stream-ordered allocator may hand them out again on the same stream.
 * `user` is passed back unchanged.  The callbacks must outlive the context.
 */
typedef struct {
    void* (*alloc)(void* user, size_t bytes, void* hip_stream);
    void (*free)(void* user, void* ptr, size_t bytes, void* hip_stream);
    void* user;
} cube_allocator;

/* Create a context for one box (Sec. II: the box's global coarse mesh and its
 * tiles of fine meshes with buffers; Sec. III-A: the coarse mesh is also the
 * cell grid of the position codec): validates the geometry, allocates the state,
 * the meshes and the workspace on the current device (through `alloc`, or
 * hipMalloc when it is NULL), builds the FFT twiddles (FP64-derived) and the
 * Green's tables (FP64).  hip_stream is a hipStream_t (NULL = the default
 * stream).  The state starts empty (all counts zero) until cube_compress or
 * cube_set_state.  Errors: CUBE_INVALID, CUBE_UNSUPPORTED, CUBE_OOM,
 * CUBE_DEVICE. */
cube_status cube_init(const cube_box_desc* desc, const cube_allocator* alloc, void* hip_stream,
                      cube_ctx** out);

/* Device bytes of a context for this descriptor, without allocating:
 * *persistent is held from cube_init to cube_destroy, *transient is the
 * largest set of temporaries one call adds on top (compress from host
 * buffers, the general compaction path, the power spectrum).  Errors as
 * cube_init's validation. */
cube_status cube_footprint(const cube_box_desc* desc, int64_t* persistent, int64_t* transient);

/* Free everything owned by the context (NULL is ignored). */
void cube_destroy(cube_ctx* ctx);

/* Encode float positions/velocities of n = n_side^3 particles in any order
 * into the compressed state (Eq. (2); velocity scale from the maximum speed
 * with the headroom).  pos[i*3+k] in spacings (wrapped periodically), vel in
 * spacings per unit time.  on_device: pointers are device (else host) memory.
 * Particles are ordered by canonical cell, stably with respect to the input
 * order; ids (if enabled) are the input indices.  Synchronises the stream. */
cube_status cube_compress(cube_ctx* ctx, const float* pos, const float* vel,
                          int64_t n, int32_t on_device);

/* Decode the state to float positions/velocities in canonical order (Eq. (2)
 * read back at the bin centres, exact; velocities u * s, or Eq. (3) with
 * CUBE_VEL_CELL_MEAN).  Same layout as cube_compress.  Synchronises. */
cube_status cube_decompress(cube_ctx* ctx, float* pos, float* vel, int64_t n,
                            int32_t on_device);

/* Advance the state by nsteps kick-drift steps of the two-level PM method
 * (Sec. II: coarse plus per-tile fine mesh force, Eq. (1); Sec. III-A: the
 * positions and velocities are requantised and the particles recounted and
 * reordered by cell after each step).  All steps are enqueued on the
 * context stream with no host synchronisation and no allocation between
 * them; every choice a step makes from its own data (the compaction path,
 * accumulator widths, spectrum formats) is taken on the device, and a step
 * that needs the host (the sorted compaction for a particle that moved more
 * than one coarse cell, or a plan change) stops the later ones until the
 * host resolves it after the one read-back at the end.  A CUBE_MIXED_FP16
 * potential spectrum value outside the FP16 range makes that step run again
 * with FP32 spectra.  Returns after the last step; errors CUBE_OOM (the
 * sorted compaction's temporaries; the state is then the one before that
 * step), CUBE_DEVICE. */
cube_status cube_pm_step(cube_ctx* ctx, int32_t nsteps);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * steps as cube_pm_step, with the only temporaries a step can need (those
 * of the sorted general compaction, 16 bytes per particle plus the sort's
 * workspace) taken from a fixed region of 36 MiB that the library holds on
 * each device for the life of the process, so no call allocates or frees.
 * Boxes above 128^3 particles (more scratch than the region) are refused
 * with CUBE_INVALID, as is a context with profiling on.  Every call on one
 * device shares that region: calls that overlap on a device (two host
 * threads, or contexts on different streams) race and must be serialised by
 * the caller.  The region needs no clearing between calls (every word is
 * written before it is read). */
cube_status cube_pm_step_noalloc(cube_ctx* ctx, int32_t nsteps);

/* Acceleration of every particle at the current state, no update: coarse
 * plus fine mesh force (Sec. II, Eq. (1)), plus the pair force when
 * pp_range > 0, in static units (the comoving kick factor is not applied).
 * acc[i*3+k], canonical order, float32.  Synchronises.  A CUBE_MIXED_FP16
 * potential spectrum value outside the FP16 range makes it evaluate again
 * with FP32 spectra. */
cube_status cube_forces(cube_ctx* ctx, float* acc, int32_t on_device);

/* Copy the state out to / in from caller buffers (see cube_state_view).
 * set_state validates that the counts sum to n_particles.  Synchronises. */
cube_status cube_get_state(cube_ctx* ctx, cube_state_view* view);
cube_status cube_set_state(cube_ctx* ctx, const cube_state_view* view);

/* FP64 diagnostics (mass, momentum, kinetic and potential energy, counters)
 * of the current state: the conserved quantities against which a PM run is
 * checked (Sec. IV-C compares the evolved matter field; mass is exact here
 * because the deposit of Sec. II is integer).  Synchronises. */
cube_status cube_diagnostics(cube_ctx* ctx, cube_diag* out);

/* Matter power spectrum of the current state (Sec. IV-C: delta = rho/rho_bar
 * - 1, P(k) and Delta^2(k) = k^3 P(k) / (2 pi^2)): CIC on a mesh of one cell per
 * spacing, delta = rho - 1, P = L^3 |DFT(delta)|^2 / N_cells^2 averaged over
 * shells j = round(|n|), 1 <= j < n_side/4.  Host arrays of nbins entries
 * (nbins must be n_side/4 - 1).  Synchronises. */
cube_status cube_power_spectrum(cube_ctx* ctx, int32_t nbins, double* k,
                                double* pk, int64_t* nmodes);

/* Test hook: write an intermediate mesh of the current state into a caller
 * device buffer of float32.  what: 0 coarse density rho_c - 1 (N_c^3),
 * 1 coarse potential (N_c^3), 2 fine density of tile `tile` (F^3),
 * 3 fine potential of tile `tile` (F^3).  Layout [z][y][x], x fastest. */
cube_status cube_debug_mesh(cube_ctx* ctx, int32_t what, int32_t tile, float* out);

/* Test hook: force a condition in the next `count` steps of cube_pm_step so
 * that the host-side recovery runs on ordinary states.  what: 1 raise the
 * FP16 range flag (the step runs again with FP32 spectra), 2 take the sorted
 * general compaction (same order as the fast one), 3 stop the steps after
 * this one for a new plan.  The results equal those of unforced steps. */
cube_status cube_debug_force(cube_ctx* ctx, int32_t what, int32_t count);

/* Utility: in-place unnormalised 3-D complex FFT of an n^3 interleaved
 * (re, im) float32 device array, [z][y][x] layout, sign -1 (inverse = 0) or
 * +1 (inverse = 1), using the library's LDS Stockham kernels.  n must factor
 * into the supported radices (CUBE_UNSUPPORTED otherwise).  hip_stream may be
 * NULL.  Synchronises. */
cube_status cube_fft3d(int32_t n, float* data, int32_t inverse, void* hip_stream);

/* Per-stage timing of cube_pm_step, measured with HIP events recorded on the
 * context stream around every launch of the stage (profiling adds one event
 * pair per launch).  `bytes` is the stage's algorithmic traffic summed over
 * its launches (what the method must move: particle bytes, mesh reads and
 * writes), so bytes / (total_ms * 1e-3) is its achieved rate. */
typedef struct {
    char name[32];
    int64_t launches;
    double total_ms;
    double bytes;
} cube_stage_stat;

/* Enable (nonzero) or disable profiling; enabling clears the counters. */
cube_status cube_profile_enable(cube_ctx* ctx, int32_t enable);

/* Copy up to max stage records into out; *n receives the number written. */
cube_status cube_profile_read(cube_ctx* ctx, cube_stage_stat* out, int32_t max, int32_t* n);

/*
 * Serving: independent boxes submitted one by one, each run to completion
 * (compress, n_steps steps, optional diagnostics and state copy-out) on one
 * GPU.  Admission is first-in first-out against an HBM budget: the request at
 * the head of the queue starts when a slot is free and its footprint
 * (persistent + transient bytes from cube_footprint) fits in what running
 * boxes leave of the budget.  Each slot is one host thread with its own HIP
 * stream and context, so up to max_slots boxes run concurrently.
 *   hbm_budget_bytes  device bytes the running boxes may hold together.
 *   max_slots         boxes in flight at once (>= 1).
 *   precision         cube_precision forced on every request, or -1 to keep
 *                     each request's own.
 *   device            HIP device of every context.
 * The server is internally synchronised: any thread may submit and poll.
 */
typedef struct {
    int64_t hbm_budget_bytes;
    int32_t max_slots;
    int32_t precision;
    int32_t device;
    int32_t reserved;
} cube_server_desc;

/*
 * One box.  pos/vel are host arrays [n][3] (as for cube_compress) and
 * out_state, if not NULL, receives the final state (host buffers, as for
 * cube_get_state).  The caller keeps all of them alive and unchanged until
 * cube_poll reports the request done.  want_diag nonzero: fill the result's
 * diagnostics (costs about one force evaluation).
 */
typedef struct {
    cube_box_desc desc;
    int32_t n_steps;
    int32_t want_diag;
    const float* pos;
    const float* vel;
    int64_t n;
    cube_state_view* out_state;
} cube_request;

/* Outcome of a request; times are milliseconds on the server's steady clock
 * (0 = cube_server_create). */
typedef struct {
    int32_t status;            /* cube_status of the run                        */
    int32_t reserved;
    int64_t steps_done;
    int64_t footprint_bytes;   /* bytes admitted against the budget            */
    double submit_ms;
    double start_ms;           /* admitted and started                          */
    double done_ms;
    cube_diag diag;            /* when want_diag                                */
    char message[160];         /* cube_last_error text of a failed run          */
} cube_result;

typedef struct cube_server cube_server;

/* Start the slot threads.  Errors: CUBE_INVALID (bad descriptor). */
cube_status cube_server_create(const cube_server_desc* desc, cube_server** out);

/* Queue a request; *ticket identifies it.  CUBE_INVALID if the descriptor
 * is invalid, the arrays are missing or n != n_side^3, or the footprint
 * exceeds the whole budget (it could never be admitted); CUBE_UNSUPPORTED as
 * for cube_init. */
cube_status cube_submit(cube_server* srv, const cube_request* req, uint64_t* ticket);

/* CUBE_NOT_READY while the request waits or runs; CUBE_OK once it is done,
 * with *out filled (the ticket is then released: polling it again is
 * CUBE_INVALID); CUBE_INVALID for an unknown ticket. */
cube_status cube_poll(cube_server* srv, uint64_t ticket, cube_result* out);

/* Wait for the running boxes, drop the queued ones, stop the threads.  NULL
 * is ignored. */
void cube_server_destroy(cube_server* srv);

/*
 * Batched ensembles: many independent boxes of different sizes advanced
 * together (the two-level PM step of Sec. II on the compressed particles of
 * Sec. III-A, box by box, with the boxes' tile work merged).  Boxes whose
 * tiles share one FFT geometry (tile box, tile side, buffer, split radius,
 * resolution, precision) share a fine workspace of `tiles_in_flight` tile
 * meshes: their tiles pass through it in waves, and each wave's three fine
 * FFT sweeps are single persistent launches over the tiles of every box in
 * the wave.  The boxes' own stages run on `streams` HIP streams (boxes
 * assigned round robin, default priority), joined around every shared FFT.
 * One ensemble step is captured into a hipGraph once and replayed; nothing
 * synchronises with the host inside a step.  Each box's result is the one it
 * gets alone (same kernels, same order of arithmetic).
 *   streams          1..4, or 0: chosen by the autotuner.
 *   tiles_in_flight  tile meshes per shared workspace, or 0: chosen by the
 *                    autotuner (the workspace is sized for up to 256 tiles,
 *                    or the largest class).
 *   use_graph        0: captured hipGraph steps (default); -1: eager launches.
 *   device           HIP device of every box.
 * Boxes must be static (comoving = 0), use the linear velocity codec and
 * CUBE_FP32 or CUBE_MIXED_BF16 (CUBE_UNSUPPORTED otherwise).
 */
typedef struct {
    int32_t streams;
    int32_t tiles_in_flight;
    int32_t use_graph;
    int32_t device;
} cube_ensemble_desc;

typedef struct cube_ensemble cube_ensemble;

/* Create the boxes (empty states, each one's own context with a one-tile
 * fine workspace) and the shared workspaces.  Errors as cube_init, and
 * CUBE_UNSUPPORTED for the box kinds above. */
cube_status cube_ensemble_create(const cube_box_desc* boxes, int32_t nboxes, const cube_ensemble_desc* opts,
                                 cube_ensemble** out);

/* Borrow box i's context for cube_compress / cube_set_state /
 * cube_get_state / cube_diagnostics (it stays owned by the ensemble; do not
 * destroy it, and do not use it while cube_ensemble_step runs). */
cube_status cube_ensemble_box(cube_ensemble* e, int32_t i, cube_ctx** out);

/* Advance every box by nsteps steps.  On the first call of an ensemble whose
 * schedule is left to the autotuner (and not yet cached for this set of box
 * geometries in the process), the tuner runs first.  A box that needs the
 * host (see cube_pm_step) finishes its steps on its own after the others. */
cube_status cube_ensemble_step(cube_ensemble* e, int32_t nsteps);

/* Autotuner: time one ensemble step of every candidate schedule (streams 1,
 * 2, 4 x tiles in flight 16, 32, ... up to the workspace) on the current
 * states, restore the states after each, keep the fastest and cache it for
 * this set of box geometries.  The chosen schedule is written to *chosen
 * when not NULL.  Only non-numerical knobs change: results are identical
 * under every schedule. */
cube_status cube_ensemble_tune(cube_ensemble* e, cube_ensemble_desc* chosen);

/* The schedule in use. */
cube_status cube_ensemble_schedule(cube_ensemble* e, cube_ensemble_desc* out);

/* Destroy the boxes, workspaces, streams and graph (NULL is ignored). */
void cube_ensemble_destroy(cube_ensemble* e);

#ifdef __cplusplus
}
#endif

#endif /* CUBE_H */
