// Host-side state of one box context and the pieces of a step, shared by
// the C ABI (api.cpp) and the ensemble runner (ensemble.cpp).  Nothing here
// crosses the C ABI.
#pragma once

#include <algorithm>
#include <cstdint>
#include <string>
#include <utility>
#include <vector>

#include "../../include/cube.h"
#include "internal.h"

namespace cube {

// Records msg as the calling thread's last error and returns st.
cube_status fail(cube_status st, const std::string& msg);

#define CUBE_HIP(expr)                                                                         \
    do {                                                                                       \
        hipError_t e_ = (expr);                                                                \
        if (e_ != hipSuccess) {                                                                \
            return fail(CUBE_DEVICE, std::string(#expr) + ": " + hipGetErrorString(e_));       \
        }                                                                                      \
    } while (0)

enum Stage {
    ST_COARSE_DEP, ST_COARSE_FFT, ST_FINE_DEP, ST_FFT_R2C, ST_FFT_ZG, ST_FFT_C2R,
    ST_GATHER, ST_SCAN, ST_COMPACT, ST_VENC, ST_PP, NSTAGES
};
// HIP events around every launch of a stage, resolved at the next sync.
struct Profiler {
    bool on = false;
    struct Pending {
        int stage;
        hipEvent_t a, b;
        double bytes;
    };
    std::vector<hipEvent_t> pool;
    std::vector<Pending> pending;
    int64_t launches[NSTAGES] = {};
    double ms[NSTAGES] = {};
    double bytes[NSTAGES] = {};

    hipEvent_t get() {
        if (pool.empty()) {
            hipEvent_t e;
            hipEventCreate(&e);
            return e;
        }
        hipEvent_t e = pool.back();
        pool.pop_back();
        return e;
    }
    hipEvent_t mark(hipStream_t s) {
        hipEvent_t e = get();
        hipEventRecord(e, s);
        return e;
    }
    void add(int stage, hipEvent_t a, hipEvent_t b, double by) { pending.push_back({stage, a, b, by}); }
    // call only after the stream has been synchronised
    void flush() {
        std::vector<hipEvent_t> done;
        for (const Pending& p : pending) {
            float t = 0.f;
            if (hipEventElapsedTime(&t, p.a, p.b) == hipSuccess) {
                ms[p.stage] += t;
                launches[p.stage] += 1;
                bytes[p.stage] += p.bytes;
            }
            done.push_back(p.a);
            done.push_back(p.b);
        }
        pending.clear();
        std::sort(done.begin(), done.end());
        done.erase(std::unique(done.begin(), done.end()), done.end());
        for (hipEvent_t e : done) pool.push_back(e);
    }
    void reset() {
        for (int i = 0; i < NSTAGES; ++i) { launches[i] = 0; ms[i] = 0.0; bytes[i] = 0.0; }
    }
    ~Profiler() {
        for (const Pending& p : pending) { hipEventDestroy(p.a); hipEventDestroy(p.b); }
        for (hipEvent_t e : pool) hipEventDestroy(e);
    }
};

inline size_t round256(size_t bytes) { return std::max<size_t>((bytes + 255) / 256 * 256, 256); }

// Device memory: the caller's callbacks, or hipMalloc / hipFree.  Sizes are
// rounded up to 256 bytes, and the same rounded size is passed to free.
struct DevMem {
    cube_allocator al{};
    bool custom = false;
    hipStream_t stream = nullptr;
    void* get(size_t bytes) {
        bytes = round256(bytes);
        if (custom) return al.alloc(al.user, bytes, stream);
        void* p = nullptr;
        if (hipMalloc(&p, bytes) != hipSuccess) {
            (void)hipGetLastError();
            return nullptr;
        }
        return p;
    }
    void put(void* p, size_t bytes) {
        if (!p) return;
        if (custom) al.free(al.user, p, round256(bytes), stream);
        else hipFree(p);
    }
};

// Buffers that live for one call; released (stream-ordered) at scope exit.
struct Temp {
    DevMem& mem;
    std::vector<std::pair<void*, size_t>> held;
    explicit Temp(DevMem& m) : mem(m) {}
    template <class T>
    bool get(T** p, size_t bytes) {
        void* q = mem.get(bytes);
        *p = static_cast<T*>(q);
        if (!q) return false;
        held.push_back({q, bytes});
        return true;
    }
    ~Temp() {
        for (auto& e : held) mem.put(e.first, e.second);
    }
};

// What the host fixes when it enqueues a step, from the state's counts as of
// its last synchronisation: the fine-deposit accumulator width and the
// storage format of the tile half spectra.  The mixed FP16 mode falls back to
// FP32 while a fine-cell density could exceed the FP16 range (a fine cell
// gathers the particles of at most one 2x2x2 block of coarse cells, density
// f^3 per particle; the plane transform's gain is divided out), and after a
// potential spectrum value left it (force_fp32).  The epilogue of every step
// checks that the new state still fits the plan (halt 3 otherwise).
struct StepPlan {
    bool wide;
    int fmt;
};

}  // namespace cube

struct cube_ctx {
    cube::Profiler prof;
    cube::Geom g{};
    cube_box_desc desc{};
    hipStream_t stream = nullptr;
    bool poisoned = false;
    bool has_state = false;
    cube::DevMem mem;
    std::vector<std::pair<void*, size_t>> allocs;

    cube::Planes A{}, B{};
    cube::VelCells vcell{};                 // cell-mean velocity codec: means and tan table
    uint8_t* dir = nullptr;
    uint32_t* far_key = nullptr;
    uint4* ment = nullptr;            // mover records, one slot per particle
    int32_t* mhdr = nullptr;          // per gather brick: first record slot and per-class offsets
    int32_t* tcursor = nullptr;       // per tile: record slots taken in the running step
    int32_t* counts = nullptr;
    int32_t* offsets = nullptr;
    int32_t* counts_new = nullptr;
    int32_t* offsets_new = nullptr;
    cube::StepScalars* sc = nullptr;
    cube::StepScalars* sc_host = nullptr;   // pinned

    float2* coarse = nullptr;
    double* coarse_green = nullptr;
    float2* tw_coarse = nullptr;
    float* fine_real = nullptr;       // batch x F^3 real meshes (density, then potential)
    void* fine_spec = nullptr;        // batch x F^2 (F/2+1) half spectra (FP32 size: FP16 may fall back)
    float* fine_green = nullptr;
    float2* tw_fine = nullptr;
    void* scan_ws = nullptr;
    double* partial = nullptr;
    double* reduced = nullptr;
    float* pp[3] = {nullptr, nullptr, nullptr};   // extended PP accelerations, [3][n]
    int batch = 1;

    int64_t step = 0;
    double last_step_ms = 0.0;
    int32_t max_count = 0;            // largest cell count of the current state
    int32_t max_block8 = 0;           // largest count of a 2x2x2 block of coarse cells
    bool halted_recently = false;     // the last cube_pm_step met a halt: enqueue one step per sync
    int dbg_force[4] = {0, 0, 0, 0};  // cube_debug_force: steps still to receive each forced condition
    void* noalloc_scratch = nullptr;  // this device's fixed scratch region (cube_pm_step_noalloc)

    ~cube_ctx() {
        if (sc_host) hipHostFree(sc_host);
        for (auto& e : allocs) mem.put(e.first, e.second);
    }

    cube_status alloc(void** p, size_t bytes) {
        *p = mem.get(bytes);
        if (!*p) return cube::fail(CUBE_OOM, "device allocation of " + std::to_string(cube::round256(bytes)) + " bytes failed");
        allocs.push_back({*p, bytes});
        return CUBE_OK;
    }
    template <class T>
    cube_status alloc_n(T** p, int64_t n) {
        return alloc(reinterpret_cast<void**>(p), (size_t)n * sizeof(T));
    }
};

namespace cube {

cube_status check_ctx(cube_ctx* c);
cube_status launch_status(cube_ctx* c);
cube_status sync(cube_ctx* c);
StepPlan plan_of(const cube_ctx* c, bool force_fp32 = false);

// One step in pieces, enqueued on c->stream with no synchronisation: the
// prologue, coarse potential and pair forces; the gather/kick/drift of tiles
// [t0, t0 + nt) from their fine potentials in `mesh` (nt real F^3 meshes);
// recount, compaction and commit.  enqueue_step runs them around the fine
// deposits and solves of the context's own meshes.
void step_pre(cube_ctx* c);
void step_gather(cube_ctx* c, int t0, int nt, const float* mesh, int64_t step_index);
void step_post(cube_ctx* c, const StepPlan& plan);
void enqueue_step(cube_ctx* c, const StepPlan& plan, int64_t step_index);
// the rows [lo, hi) of a tile box that the fine solve must write for the gather
void fine_window(const Geom& g, bool full, int* lo, int* hi);

// Wait for the enqueued work and read the step scalars back.
cube_status read_scalars(cube_ctx* c);
// Resolve the halt a context stopped at (after read_scalars; base_done is
// its committed step count when the halted step began): finish a general
// compaction, or clear a halt for an FP16 overflow (*force_fp32 is then set)
// or a re-plan.  Steps committed here are added to c->step.
cube_status resolve_halt(cube_ctx* c, void* scratch, bool* force_fp32, int64_t base_done);
// nsteps steps: enqueue, read back once, resolve halts, continue.
cube_status run_steps(cube_ctx* c, int32_t nsteps, void* scratch);

}  // namespace cube
