// Internal declarations shared by the host orchestration and the kernels of
// libcube.so.  Nothing here crosses the C ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>
#include <cstddef>

namespace cube {

// Sets the calling thread's message returned by cube_last_error().
void set_last_error(const char* msg);

// Box geometry in the integer units the kernels use (Sec. II tiles + buffers,
// Sec. III-A coarse-cell codec).  All sides are cell counts.
struct Geom {
    int ns;        // particles per side
    int f;         // fine cells per spacing
    int r;         // fine cells per coarse cell
    int nt;        // tiles per side
    int b;         // buffer, fine cells
    int a;         // split radius, fine cells
    int Nc;        // coarse cells per side
    int T;         // tile side, fine cells
    int Tc;        // tile side, coarse cells
    int F;         // tile FFT box side, fine cells
    int Fc;        // tile FFT box side, coarse cells (F / r)
    int hc;        // buffer in coarse cells (b / r)
    int log2D;     // log2(512 / r): fine-coordinate fraction bits
    int periodic;  // 1 when the single tile is the periodic box
    int fdr;       // reach of the gradient stencil: 1 (2-point) or 2 (4-point)
    int vcodec;    // velocity storage: 0 linear bytes, 1 cell means + Eq. (3) bytes
    int npp;       // extended PP range in fine cells (0: off)
    int64_t ncells;   // Nc^3
    int64_t n;        // ns^3 particles
    int ntiles;       // nt^3
    int tc_shift;     // log2(Tc) when Tc is a power of two, else -1
    int nt_shift;     // log2(nt) when nt is a power of two, else -1
};

// Canonical cell index: tile-major (tile index x fastest), x fastest inside.
__host__ __device__ inline int64_t canon(const Geom& g, int cx, int cy, int cz) {
    if (g.tc_shift >= 0 && g.nt_shift >= 0) {
        const int s = g.tc_shift, m = g.Tc - 1, ns = g.nt_shift;
        const int64_t tile = (cx >> s) + ((int64_t)((cy >> s) + ((cz >> s) << ns)) << ns);
        return (tile << (3 * s)) + (cx & m) + ((int64_t)((cy & m) + ((cz & m) << s)) << s);
    }
    int tx = cx / g.Tc, ty = cy / g.Tc, tz = cz / g.Tc;
    int lx = cx - tx * g.Tc, ly = cy - ty * g.Tc, lz = cz - tz * g.Tc;
    int64_t tile = tx + (int64_t)g.nt * (ty + (int64_t)g.nt * tz);
    return tile * ((int64_t)g.Tc * g.Tc * g.Tc) + lx + (int64_t)g.Tc * (ly + (int64_t)g.Tc * lz);
}

__host__ __device__ inline int wrapi(int x, int n) {
    int m = x % n;
    return m < 0 ? m + n : m;
}

// Per-step scalars that live on the device so that nothing syncs mid-step.
// A step's kernels that write the state or these scalars return at once
// while `halt` is set; the host resolves a halt at its next synchronisation:
//   1  the step needs the sorted general compaction (a particle moved more
//      than one coarse cell, or a cell count exceeds the fast path's bound);
//      everything up to the compaction is done and kept for it;
//   2  a CUBE_MIXED_FP16 potential spectrum value left the FP16 range; the
//      step is run again with FP32 spectra;
//   3  the new state needs a wider fine-deposit accumulator or FP32 density
//      spectra than the host planned for the next step; the step itself is
//      complete, the following ones are enqueued again.
struct StepScalars {
    // read by every block of a step's kernels; kept off the lines that the
    // per-block atomics below update, or each read queues behind them
    int32_t halt;        // see above; 0 while steps run normally
    int32_t pad_[63];
    double s;            // velocity scale of the state
    double s_next;       // scale after the coming kick
    int32_t max_u;       // max |u| of the state
    int32_t max_u_next;  // accumulated by the kick
    int32_t far_count;   // particles whose carry exceeds one cell
    int32_t max_carry;   // max |carry| of the step
    int64_t saturations; // clamped velocity components (cumulative, committed by the epilogue)
    int64_t sat_step;    // clamped components of the running step
    int32_t overflow;    // a 16-bit spectrum value was out of range (cleared by the prologue)
    int32_t max_count;   // largest cell count of the state
    int32_t max_block8;  // largest count of a 2x2x2 block of coarse cells of the state
    int32_t new_max_count;   // the same two of the step's new counts (set by the scan, adjacent)
    int32_t new_max_block8;
    int64_t steps_done;  // steps committed since the context was made
    // per-block maxima land in 64 slots (spreads atomic contention); the
    // epilogue folds them into max_u / max_carry
    int32_t umax_slot[64];
    int32_t cmax_slot[64];
};

// Particle planes: m[3] uint8 then u[3] int8, each of capacity n; with the
// cell-mean velocity codec also FP32 working velocities v[3] (else null).
// Copies (compaction, permutation) move every non-null plane.
struct Planes {
    uint8_t* m[3];
    int8_t* u[3];
    uint32_t* ids;   // may be null
    float* v[3];     // may be null
};

// Cell-mean velocity codec state: FP32 mean velocity per axis and coarse cell
// (canonical order) and the FP64 table tan(u pi / 255), u = -127..127.
struct VelCells {
    float* vc[3];
    const double* tab;
};

// ---- scan.hip -----------------------------------------------------------
// out[0..n] = exclusive prefix sum of in[0..n-1]; out[n] = total.  If max_out
// is given, atomicMax(max_out, max(in)) as well.
size_t scan_workspace_bytes(int64_t n);
// gate (optional): every kernel returns at once while *gate is nonzero.
void exclusive_scan_i32(const int32_t* in, int32_t* out, int64_t n, void* ws, hipStream_t s,
                        int32_t* max_out = nullptr, const int32_t* gate = nullptr);
// out[0] += 64-bit sum of counts[0..n), out[1] = min(out[1], smallest count)
// (out[0] = 0 and out[1] = INT64_MAX on entry)
void launch_count_check(const int32_t* counts, int64_t n, long long* out, hipStream_t s);

// ---- sort.hip -----------------------------------------------------------
// Stable LSD sort of (key, value) pairs by the low `bits` key bits.
size_t sort_workspace_bytes(int64_t n);
void stable_sort_pairs(uint32_t* key, uint32_t* val, uint32_t* key_tmp, uint32_t* val_tmp,
                       int64_t n, int bits, void* ws, hipStream_t s);

// ---- codec.hip ----------------------------------------------------------
void launch_encode_keys(const Geom& g, const float* pos, uint32_t* key, uint32_t* qpack,
                        uint32_t* idx, int64_t n, hipStream_t s);
void launch_absmax_f32(const float* v, int64_t n, uint32_t* out_bits, hipStream_t s);
void launch_scatter_compressed(const Geom& g, const uint32_t* perm, const uint32_t* qpack,
                               const float* vel, double s_v, Planes out, int32_t* counts,
                               StepScalars* sc, int64_t n, hipStream_t st);
void launch_decode(const Geom& g, const int32_t* offsets, Planes in, const StepScalars* sc,
                   const VelCells& vcell, float* pos, float* vel, hipStream_t s);
void launch_count_keys(const uint32_t* key, int64_t n, int32_t* counts, hipStream_t s);

// ---- vcodec.hip ---------------------------------------------------------
// Cell-mean velocity codec (Eq. (3), Eq. (4)) on the FP32 velocities p.v of
// a cell-ordered state: cell means into vcell.vc, sigma into sc->s, codes
// into p.u; saturated components are added to sc->saturations and max |u|
// replaces sc->max_u.  partial: vc_partials(g) doubles of workspace.
void vc_table_host(double* tab255);
int vc_partials(const Geom& g);
void launch_vc_encode(const Geom& g, const int32_t* offsets, Planes p, const VelCells& vcell,
                      StepScalars* sc, double* partial, hipStream_t s, bool gated = false);

// ---- deposit.hip --------------------------------------------------------
void launch_coarse_deposit(const Geom& g, const int32_t* offsets, Planes p, float2* mesh,
                           int32_t* overflow, hipStream_t s);
// real density meshes of tiles [tile0, tile0 + ntiles) into mesh + k F^3;
// wide selects 64-bit accumulators (needed when fine_deposit_needs_wide)
void launch_fine_deposit(const Geom& g, const int32_t* offsets, Planes p, int tile0, int ntiles,
                         float* mesh, bool wide, hipStream_t s);
bool fine_deposit_needs_wide(const Geom& g, int max_block8);
bool fp16_density_fits(const Geom& g, int max_block8);
// atomicMax(*out, largest count of a periodic 2 x 2 x 2 block of coarse cells)
void launch_max_block8(const Geom& g, const int32_t* counts, int32_t* out, hipStream_t s,
                       const int32_t* gate = nullptr);
void launch_diag_deposit(const Geom& g, const int32_t* offsets, Planes p, float2* mesh,
                         hipStream_t s);

// ---- fft.hip ------------------------------------------------------------
bool fft_supported(int n);
// Twiddle table exp(-2 pi i k / n), FP64-derived, n entries (device memory).
void fft_make_twiddles(int n, float2* dev_table, hipStream_t s);
// Forward or inverse 3-D transform of `batch` cubes of side n.
void fft3d(float2* data, int n, int batch, bool inverse, const float2* tw, hipStream_t s);
// Forward 3-D, multiply by a real octant Green's table, inverse 3-D.
// table_kind: 0 = float octant (n/2+1)^3, 1 = double octant.
// ev (optional, 6 events): recorded before the first pass and after each pass.
void fft3d_convolve(float2* data, int n, int batch, const float2* tw, const void* green_octant,
                    int table_kind, hipStream_t s, hipEvent_t* ev = nullptr);

// Real tile meshes (ntiles cubes of n^3 floats, [z][y][x]) -> convolution with
// a real even octant table (pencil-major, as build_fine_green writes it) through half spectra (n^2 (n/2+1) complex per
// tile, workspace) -> potentials in place.  spec_format: 0 FP32 complex,
// 1 BF16 pairs, 2 scaled FP16 pairs (4 bytes per complex value); with FP16 an
// out-of-range value sets *range_flag = 1.  Only the window [out_lo, out_hi)^3
// of each potential is written (the rest of the real mesh keeps the density).
// ev (optional, 4 events) is recorded before the first and after each of the
// three sweeps.
bool fft_tiles_supported(int n);
void fft_tiles_convolve(float* real_tiles, void* spec_tiles, int n, int ntiles, const float2* tw,
                        const float* green_octant, int spec_format, int32_t* range_flag, int out_lo, int out_hi,
                        hipStream_t s, hipEvent_t* ev = nullptr);

// ---- green.hip ----------------------------------------------------------
// Octant tables computed in FP64, already divided by n^3 (the inverse-FFT
// normalisation): coarse FP64 [kz][ky][kx]; fine rounded to FP32 and stored
// pencil-major [ky][kx][kz] for the z-pencil pass.
void build_coarse_green(const Geom& g, double* octant, hipStream_t s);
void build_fine_green(const Geom& g, float* octant, void* ws, hipStream_t s);
size_t fine_green_workspace_bytes(const Geom& g);

// ---- gather bricks --------------------------------------------------------
// The gather and the compaction share one decomposition: bricks of 32 x 16 x 8
// fine cells, whole coarse cells (r = 4 or 8), numbered tile-major (tile,
// then x fastest).  Each brick's header holds kHdrInts ints: the first slot
// of its mover records, then for the 27 classes of destination brick
// (dx + 1) + 3 (dy + 1) + 9 (dz + 1) the offset of the class's records and
// at [28] their total.
constexpr int kGBX = 32, kGBY = 16, kGBZ = 8;
constexpr int kHdrInts = 32;

// ---- gather.hip ---------------------------------------------------------
// floats allocated after the last fine mesh of a batch: the gather stages
// rows as aligned float2s and may read one float past a row's end
constexpr int kFineRealPad = 16;
enum GatherMode { GATHER_STEP = 0, GATHER_FORCE = 1, GATHER_POTENTIAL = 2 };
struct GatherArgs {
    Geom g;
    const int32_t* offsets;
    Planes in;
    Planes out;             // GATHER_STEP: updated m', u' at the same index
    uint8_t* dir;           // GATHER_STEP: move code 0..26, 255 = far mover
    uint32_t* far_key;      // GATHER_STEP: new canonical cell of far movers
    int32_t* counts_new;    // GATHER_STEP: histogram of new cells
    const float* fine_real;    // fine potentials of the batch: ntiles real F^3 meshes
    const float2* coarse;      // coarse potential (real part)
    StepScalars* sc;
    VelCells vcell;         // GATHER_STEP with the cell-mean codec
    const float* pp[3];     // GATHER_STEP / GATHER_FORCE: PP accelerations to add (null: none)
    float* acc;             // GATHER_FORCE: [n][3]
    double* partial;        // GATHER_POTENTIAL: per-block partial sums
    uint4* ment;            // GATHER_STEP: mover records (one slot per particle, see compact.hip)
    int32_t* mhdr;          // GATHER_STEP: per brick, kHdrInts ints (see the brick decomposition)
    int32_t* tcursor;       // GATHER_STEP: next free record slot of each tile's region (its first particle's
                            // old index at the step's start)
    double kick;            // GATHER_STEP: force multiplier of the kick (dt, or K_n comoving)
    float drift;            // GATHER_STEP: velocity multiplier of the drift (dt, or FP32 D_n)
    int tile0;
    int ntiles;
    int mode;
};
void launch_gather(const GatherArgs& a, hipStream_t s);
int gather_blocks_per_tile(const Geom& g);
bool gather_supported(const Geom& g);

// ---- pp.hip -------------------------------------------------------------
// PP accelerations of every particle of the state, [3][n] FP32 planes.
void launch_pp(const Geom& g, const int32_t* offsets, Planes in, float* const acc[3], hipStream_t s);

// ---- compact.hip --------------------------------------------------------
// fast path: the brick compaction from the gather's mover records (returns at
// once while sc->halt is set)
int64_t compact_bricks(const Geom& g);
void launch_compact_bricks(const Geom& g, const int32_t* offsets_old, const int32_t* offsets_new,
                           const uint8_t* dir, const uint4* ment, const int32_t* mhdr, Planes src, Planes dst,
                           const StepScalars* sc, hipStream_t s);
void launch_general_keys(const Geom& g, const int32_t* offsets_old, const uint8_t* dir,
                         const uint32_t* far_key, uint32_t* key, uint32_t* idx, hipStream_t s);
void launch_permute_planes(const uint32_t* perm, Planes src, Planes dst, int64_t n, hipStream_t s);

// ---- step.hip -----------------------------------------------------------
// Prologue, decision, commit and epilogue of a step: all return at once while
// sc->halt is set (the epilogue may set it, 3, after committing).
void launch_step_prologue(StepScalars* sc, float v_headroom, hipStream_t s);
// halt 2 on a spectrum overflow, else 1 when the fast compaction cannot run
// (a far mover, or a cell count above fast_max_count in the old or new counts)
void launch_step_decide(StepScalars* sc, int32_t fast_max_count, hipStream_t s);
// counts <- counts_new, offsets <- offsets_new (ncells + 1 entries)
void launch_commit_cells(const int32_t* counts_new, const int32_t* offsets_new, int32_t* counts, int32_t* offsets,
                         int64_t ncells, const StepScalars* sc, hipStream_t s);
// commit the scalars (s and max |u| only when vcodec == 0: the re-encode of
// the cell-mean codec has set them); then halt 3 if the new state escapes the
// plan of the next step (planned_wide: 64-bit fine-deposit accumulators;
// planned_f16: FP16 density spectra)
void launch_step_epilogue(StepScalars* sc, const Geom& g, int vcodec, bool planned_wide, bool planned_f16,
                          hipStream_t s);
void launch_fill_i32(int32_t* p, int32_t v, int64_t n, hipStream_t s, const int32_t* gate = nullptr);
// out[i] = in[i * stride], i < n
void launch_strided_copy(const int32_t* in, int64_t stride, int32_t* out, int64_t n, hipStream_t s,
                         const int32_t* gate = nullptr);
void launch_moments(const Geom& g, const int32_t* offsets, Planes p, const StepScalars* sc,
                    const VelCells& vcell, double* partial, int nblocks, hipStream_t s);
void launch_reduce_partials(const double* partial, int nblocks, int width, double* out,
                            hipStream_t s);
void launch_power_bins(const float2* dk, int n, int nbins, double* partial, int nparts,
                       hipStream_t s);

}  // namespace cube
