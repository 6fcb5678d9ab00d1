// Batched ensembles of independent boxes (the batched form of the two-level
// PM step of Sec. II on the compressed particles of Sec. III-A).
//
// Boxes whose tiles share one FFT geometry (tile box F, tile side T, buffer,
// split radius, resolution, precision) form a class.  A class owns one fine
// workspace of W tile meshes; the boxes' tiles pass through it in waves, and
// each wave's three fine FFT sweeps are single persistent launches over the
// tiles of every box in the wave (the plane kernels walk all planes of the
// workspace), so small boxes fill the GPU together.  The per-box stages
// (prologue, coarse mesh, fine deposits into the workspace, gathers,
// recount, compaction, commit) run on up to four HIP streams, boxes assigned
// round robin, joined around every shared FFT.  One ensemble step is
// captured into a hipGraph and replayed; a step never synchronises with the
// host, and a box that halts (see StepScalars) is resolved on its own after
// the replays.  An autotuner times candidate schedules (streams, tiles in
// flight) on the current states, which it restores afterwards, and caches
// the best per set of box geometries.
#include <chrono>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <new>

#include "ctx.h"

using namespace cube;

namespace {

constexpr int kMaxStreams = 4;

struct TileClass {
    // geometry key
    int F, T, b, f, r, a, npp, fdr, fmt, periodic;
    int lo = 0, hi = 0;                    // window the inverse sweeps write
    std::vector<std::pair<int, int>> items;   // (box, tile), box-major
    float* real = nullptr;                 // W real F^3 meshes (+ pad)
    void* spec = nullptr;                  // W half spectra (FP32 size)
    size_t real_bytes = 0, spec_bytes = 0;
};

struct Schedule {
    int streams = 0;
    int tiles = 0;     // tiles in flight per class
};

std::mutex g_tune_mu;
std::map<std::string, Schedule> g_tuned;   // geometry signature -> chosen schedule

}  // namespace

struct cube_ensemble {
    int device = 0;
    std::vector<cube_ctx*> boxes;
    std::vector<hipStream_t> streams;      // kMaxStreams created, `sched.streams` used
    std::vector<TileClass> classes;
    Schedule sched;
    bool auto_streams = false, auto_tiles = false, use_graph = true, tuned = false;
    int max_tiles = 0;                     // workspace capacity per class (tiles)
    std::vector<hipEvent_t> events;
    size_t next_event = 0;
    hipGraphExec_t exec = nullptr;
    std::vector<StepPlan> plans;           // per box, fixed in the captured graph
    std::string signature;

    hipEvent_t event() {
        if (next_event == events.size()) {
            hipEvent_t e;
            if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) return nullptr;
            events.push_back(e);
        }
        return events[next_event++];
    }
    hipStream_t stream_of(int box) const { return streams[box % sched.streams]; }

    ~cube_ensemble() {
        if (exec) hipGraphExecDestroy(exec);
        for (hipStream_t s : streams) hipStreamSynchronize(s);
        for (cube_ctx* c : boxes) cube_destroy(c);
        for (TileClass& k : classes) {
            if (k.real) hipFree(k.real);
            if (k.spec) hipFree(k.spec);
        }
        for (hipEvent_t e : events) hipEventDestroy(e);
        for (hipStream_t s : streams) hipStreamDestroy(s);
    }
};

namespace {

int spec_fmt_of(const cube_box_desc& d) { return d.precision == CUBE_MIXED_BF16 ? 1 : 0; }

// s_dst waits for everything enqueued so far on s_src
cube_status join(cube_ensemble* e, hipStream_t s_src, hipStream_t s_dst) {
    if (s_src == s_dst) return CUBE_OK;
    hipEvent_t ev = e->event();
    if (!ev || hipEventRecord(ev, s_src) != hipSuccess || hipStreamWaitEvent(s_dst, ev, 0) != hipSuccess)
        return fail(CUBE_DEVICE, "ensemble: stream join failed");
    return CUBE_OK;
}

cube_status join_all_into(cube_ensemble* e, hipStream_t s0) {
    for (int i = 0; i < e->sched.streams; ++i) {
        cube_status st = join(e, e->streams[i], s0);
        if (st != CUBE_OK) return st;
    }
    return CUBE_OK;
}

cube_status fork_from(cube_ensemble* e, hipStream_t s0) {
    for (int i = 0; i < e->sched.streams; ++i) {
        cube_status st = join(e, s0, e->streams[i]);
        if (st != CUBE_OK) return st;
    }
    return CUBE_OK;
}

// Enqueue one ensemble step (no synchronisation, no allocation).
cube_status enqueue_ensemble_step(cube_ensemble* e) {
    hipStream_t s0 = e->streams[0];
    e->next_event = 0;
    for (size_t i = 0; i < e->boxes.size(); ++i) e->boxes[i]->stream = e->stream_of((int)i);
    cube_status st = fork_from(e, s0);
    if (st != CUBE_OK) return st;
    for (cube_ctx* c : e->boxes) step_pre(c);
    for (TileClass& k : e->classes) {
        const int64_t F3 = (int64_t)k.F * k.F * k.F;
        const int W = std::min<int>(e->sched.tiles, e->max_tiles);
        for (size_t w0 = 0; w0 < k.items.size(); w0 += W) {
            const size_t w1 = std::min(k.items.size(), w0 + (size_t)W);
            // deposits of this wave's tiles into consecutive workspace slots,
            // one launch per run of consecutive tiles of one box
            for (size_t i = w0; i < w1;) {
                const int box = k.items[i].first, t0 = k.items[i].second;
                size_t j = i + 1;
                while (j < w1 && k.items[j].first == box && k.items[j].second == t0 + (int)(j - i)) ++j;
                cube_ctx* c = e->boxes[box];
                launch_fine_deposit(c->g, c->offsets, c->A, t0, (int)(j - i), k.real + (int64_t)(i - w0) * F3,
                                    e->plans[box].wide, c->stream);
                i = j;
            }
            st = join_all_into(e, s0);
            if (st != CUBE_OK) return st;
            cube_ctx* c0 = e->boxes[k.items[w0].first];
            // the FP16 range flag cannot be raised: ensembles store FP32 or BF16 spectra
            fft_tiles_convolve(k.real, k.spec, k.F, (int)(w1 - w0), c0->tw_fine, c0->fine_green, k.fmt,
                               &c0->sc->overflow, k.lo, k.hi, s0);
            st = fork_from(e, s0);
            if (st != CUBE_OK) return st;
            for (size_t i = w0; i < w1;) {
                const int box = k.items[i].first, t0 = k.items[i].second;
                size_t j = i + 1;
                while (j < w1 && k.items[j].first == box && k.items[j].second == t0 + (int)(j - i)) ++j;
                cube_ctx* c = e->boxes[box];
                step_gather(c, t0, (int)(j - i), k.real + (int64_t)(i - w0) * F3, c->step);
                i = j;
            }
            // the next wave reuses the workspace: every gather of this one first
            st = join_all_into(e, s0);
            if (st != CUBE_OK) return st;
            st = fork_from(e, s0);
            if (st != CUBE_OK) return st;
        }
    }
    for (size_t i = 0; i < e->boxes.size(); ++i) step_post(e->boxes[i], e->plans[i]);
    return join_all_into(e, s0);
}

void drop_graph(cube_ensemble* e) {
    if (e->exec) {
        hipGraphExecDestroy(e->exec);
        e->exec = nullptr;
    }
}

cube_status capture(cube_ensemble* e) {
    drop_graph(e);
    hipStream_t s0 = e->streams[0];
    if (hipStreamBeginCapture(s0, hipStreamCaptureModeThreadLocal) != hipSuccess)
        return fail(CUBE_DEVICE, "ensemble: stream capture could not begin");
    cube_status st = enqueue_ensemble_step(e);
    hipGraph_t graph = nullptr;
    const hipError_t ec = hipStreamEndCapture(s0, &graph);
    if (st != CUBE_OK) {
        if (graph) hipGraphDestroy(graph);
        return st;
    }
    if (ec != hipSuccess || !graph) return fail(CUBE_DEVICE, "ensemble: stream capture failed");
    const hipError_t ei = hipGraphInstantiate(&e->exec, graph, nullptr, nullptr, 0);
    hipGraphDestroy(graph);
    if (ei != hipSuccess) {
        e->exec = nullptr;
        return fail(CUBE_DEVICE, "ensemble: graph instantiation failed");
    }
    return CUBE_OK;
}

cube_status sync_all(cube_ensemble* e) {
    for (hipStream_t s : e->streams)
        if (hipStreamSynchronize(s) != hipSuccess) return fail(CUBE_DEVICE, "ensemble: stream synchronisation failed");
    return CUBE_OK;
}

// Per-box plans from the states as of the last synchronisation; the graph is
// stale when one changed.
bool refresh_plans(cube_ensemble* e) {
    bool changed = e->plans.size() != e->boxes.size();
    e->plans.resize(e->boxes.size());
    for (size_t i = 0; i < e->boxes.size(); ++i) {
        const StepPlan p = plan_of(e->boxes[i]);
        if (p.wide != e->plans[i].wide || p.fmt != e->plans[i].fmt) changed = true;
        e->plans[i] = p;
    }
    return changed;
}

// nsteps ensemble steps; a box that halted finishes its steps on its own.
cube_status run_ensemble(cube_ensemble* e, int32_t nsteps) {
    if (nsteps <= 0) return CUBE_OK;
    cube_status st = sync_all(e);
    if (st != CUBE_OK) return st;
    for (cube_ctx* c : e->boxes) {
        st = read_scalars(c);
        if (st != CUBE_OK) return st;
    }
    if (refresh_plans(e)) drop_graph(e);
    std::vector<int64_t> base(e->boxes.size());
    for (size_t i = 0; i < e->boxes.size(); ++i) base[i] = e->boxes[i]->sc_host->steps_done;
    hipStream_t s0 = e->streams[0];
    if (e->use_graph) {
        if (!e->exec) {
            st = capture(e);
            if (st != CUBE_OK) return st;
        }
        for (int32_t k = 0; k < nsteps; ++k)
            if (hipGraphLaunch(e->exec, s0) != hipSuccess) return fail(CUBE_DEVICE, "ensemble: graph launch failed");
    } else {
        for (int32_t k = 0; k < nsteps; ++k) {
            st = enqueue_ensemble_step(e);
            if (st != CUBE_OK) return st;
            for (cube_ctx* c : e->boxes) c->step += 1;
        }
        for (cube_ctx* c : e->boxes) c->step -= nsteps;
    }
    st = sync_all(e);
    if (st != CUBE_OK) return st;
    for (size_t i = 0; i < e->boxes.size(); ++i) {
        cube_ctx* c = e->boxes[i];
        c->stream = e->stream_of((int)i);
        st = read_scalars(c);
        if (st != CUBE_OK) return st;
        const int64_t done = c->sc_host->steps_done - base[i];
        c->step += done;
        if (c->sc_host->halt != 0) {
            bool force_fp32 = false;
            const int64_t before = c->step;
            st = resolve_halt(c, nullptr, &force_fp32, base[i] + done);
            if (st != CUBE_OK) return st;
            const int64_t left = nsteps - done - (c->step - before);
            if (left > 0) {
                st = run_steps(c, (int32_t)left, nullptr);
                if (st != CUBE_OK) return st;
            }
            drop_graph(e);
        } else if (done != nsteps) {
            return fail(CUBE_DEVICE, "ensemble: a box committed fewer steps than launched");
        }
    }
    return CUBE_OK;
}

// Device copies of every box's state and step scalars, for the tuner.
struct Snapshot {
    std::vector<void*> bufs;
    std::vector<StepScalars> sc;
    std::vector<int64_t> step;
    ~Snapshot() {
        for (void* p : bufs)
            if (p) hipFree(p);
    }
};

size_t state_bytes(const cube_ctx* c) {
    const size_t n = (size_t)c->g.n, cells = (size_t)c->g.ncells;
    return 6 * n + (c->A.ids ? 4 * n : 0) + 4 * cells + 4 * (cells + 1);
}

cube_status copy_state(cube_ctx* c, char* buf, bool save) {
    const size_t n = (size_t)c->g.n, cells = (size_t)c->g.ncells;
    hipStream_t s = c->stream;
    auto mv = [&](void* dev, size_t bytes, size_t& off) {
        const hipError_t er = save ? hipMemcpyAsync(buf + off, dev, bytes, hipMemcpyDeviceToDevice, s)
                                   : hipMemcpyAsync(dev, buf + off, bytes, hipMemcpyDeviceToDevice, s);
        off += bytes;
        return er == hipSuccess;
    };
    size_t off = 0;
    bool ok = true;
    for (int k = 0; k < 3; ++k) {
        ok = ok && mv(c->A.m[k], n, off);
        ok = ok && mv(c->A.u[k], n, off);
    }
    if (c->A.ids) ok = ok && mv(c->A.ids, 4 * n, off);
    ok = ok && mv(c->counts, 4 * cells, off);
    ok = ok && mv(c->offsets, 4 * (cells + 1), off);
    return ok ? CUBE_OK : fail(CUBE_DEVICE, "ensemble: state copy failed");
}

cube_status snapshot(cube_ensemble* e, Snapshot& snap, bool save) {
    cube_status st = sync_all(e);
    if (st != CUBE_OK) return st;
    if (save) {
        snap.bufs.assign(e->boxes.size(), nullptr);
        snap.sc.resize(e->boxes.size());
        snap.step.resize(e->boxes.size());
    }
    for (size_t i = 0; i < e->boxes.size(); ++i) {
        cube_ctx* c = e->boxes[i];
        c->stream = e->stream_of((int)i);
        if (save) {
            if (hipMalloc(&snap.bufs[i], state_bytes(c)) != hipSuccess) {
                (void)hipGetLastError();
                return fail(CUBE_OOM, "ensemble tuner: state snapshot");
            }
            st = read_scalars(c);
            if (st != CUBE_OK) return st;
            snap.sc[i] = *c->sc_host;
            snap.step[i] = c->step;
        }
        st = copy_state(c, static_cast<char*>(snap.bufs[i]), save);
        if (st != CUBE_OK) return st;
        if (!save) {
            *c->sc_host = snap.sc[i];
            if (hipMemcpyAsync(c->sc, c->sc_host, sizeof(StepScalars), hipMemcpyHostToDevice, c->stream) !=
                hipSuccess)
                return fail(CUBE_DEVICE, "ensemble tuner: scalar restore failed");
            c->step = snap.step[i];
            c->max_count = snap.sc[i].max_count;
            c->max_block8 = snap.sc[i].max_block8;
        }
    }
    return sync_all(e);
}

// Time one ensemble step of schedule `sc` (a warm step first), states restored.
cube_status time_schedule(cube_ensemble* e, const Schedule& sc, Snapshot& snap, double* ms) {
    e->sched = sc;
    drop_graph(e);
    double best = 1e300;
    for (int rep = 0; rep < 2; ++rep) {
        auto t0 = std::chrono::steady_clock::now();
        cube_status st = run_ensemble(e, 1);
        auto t1 = std::chrono::steady_clock::now();
        if (st != CUBE_OK) return st;
        st = snapshot(e, snap, false);
        if (st != CUBE_OK) return st;
        if (rep > 0) best = std::min(best, std::chrono::duration<double, std::milli>(t1 - t0).count());
    }
    *ms = best;
    return CUBE_OK;
}

cube_status tune(cube_ensemble* e, cube_ensemble_desc* report) {
    Snapshot snap;
    cube_status st = snapshot(e, snap, true);
    if (st != CUBE_OK) return st;
    const Schedule keep = e->sched;
    Schedule best = keep;
    double best_ms = 1e300;
    std::vector<int> stream_opts = e->auto_streams ? std::vector<int>{1, 2, 4} : std::vector<int>{keep.streams};
    std::vector<int> tile_opts;
    if (e->auto_tiles) {
        for (int w = 16; w <= e->max_tiles; w *= 2) tile_opts.push_back(w);
        if (tile_opts.empty() || tile_opts.back() != e->max_tiles) tile_opts.push_back(e->max_tiles);
    } else {
        tile_opts.push_back(keep.tiles);
    }
    for (int ns : stream_opts)
        for (int w : tile_opts) {
            double ms = 0.0;
            st = time_schedule(e, Schedule{ns, w}, snap, &ms);
            if (st != CUBE_OK) return st;
            if (ms < best_ms) {
                best_ms = ms;
                best = Schedule{ns, w};
            }
        }
    e->sched = best;
    drop_graph(e);
    e->tuned = true;
    {
        std::lock_guard<std::mutex> lock(g_tune_mu);
        g_tuned[e->signature] = best;
    }
    if (report) {
        report->streams = best.streams;
        report->tiles_in_flight = best.tiles;
    }
    return CUBE_OK;
}

std::string signature_of(const std::vector<cube_box_desc>& descs) {
    std::vector<std::string> parts;
    for (const cube_box_desc& d : descs) {
        char buf[160];
        std::snprintf(buf, sizeof(buf), "%d/%d/%d/%d/%d/%d/%d/%d/%d", d.n_side, d.tiles_per_dim, d.fine_per_spacing,
                      d.coarse_ratio, d.buffer_fine, d.r_cut_fine, d.fd_order, d.pp_range, d.precision);
        parts.push_back(buf);
    }
    std::sort(parts.begin(), parts.end());
    std::string s;
    for (const std::string& p : parts) s += p + ";";
    return s;
}

}  // namespace

extern "C" {

cube_status cube_ensemble_create(const cube_box_desc* descs, int32_t nboxes, const cube_ensemble_desc* opts,
                                 cube_ensemble** out) {
    if (!out) return fail(CUBE_INVALID, "null output pointer");
    *out = nullptr;
    if (!descs || nboxes <= 0) return fail(CUBE_INVALID, "an ensemble needs at least one box");
    cube_ensemble_desc o{};
    if (opts) o = *opts;
    if (o.streams < 0 || o.streams > kMaxStreams) return fail(CUBE_INVALID, "streams must be in [0, 4]");
    if (o.tiles_in_flight < 0) return fail(CUBE_INVALID, "tiles_in_flight must be >= 0");
    std::vector<cube_box_desc> ds(descs, descs + nboxes);
    for (cube_box_desc& d : ds) {
        if (d.comoving) return fail(CUBE_UNSUPPORTED, "ensembles run static boxes (comoving factors are per step)");
        if (d.vel_codec != CUBE_VEL_LINEAR) return fail(CUBE_UNSUPPORTED, "ensembles use the linear velocity codec");
        if (d.precision == CUBE_MIXED_FP16)
            return fail(CUBE_UNSUPPORTED, "ensembles store FP32 or BF16 spectra (FP16 needs a per-box range flag)");
        d.tiles_per_batch = 1;        // the boxes' own fine meshes serve only single-box calls
    }
    if (hipSetDevice(o.device) != hipSuccess) return fail(CUBE_INVALID, "bad device");
    cube_ensemble* e = new (std::nothrow) cube_ensemble();
    if (!e) return fail(CUBE_OOM, "host allocation failed");
    e->device = o.device;
    e->use_graph = o.use_graph >= 0;     // 0 (default) or 1: graphs; -1: eager launches
    for (int i = 0; i < kMaxStreams; ++i) {
        hipStream_t s;
        if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) {
            delete e;
            return fail(CUBE_DEVICE, "ensemble: stream creation failed");
        }
        e->streams.push_back(s);
    }
    e->signature = signature_of(ds);
    Schedule cached{};
    bool have_cached = false;
    {
        std::lock_guard<std::mutex> lock(g_tune_mu);
        auto it = g_tuned.find(e->signature);
        if (it != g_tuned.end()) {
            cached = it->second;
            have_cached = true;
        }
    }
    e->auto_streams = o.streams == 0;
    e->auto_tiles = o.tiles_in_flight == 0;
    e->sched.streams = o.streams ? o.streams : (have_cached ? cached.streams : kMaxStreams);
    e->tuned = have_cached || (!e->auto_streams && !e->auto_tiles);
    for (int i = 0; i < nboxes; ++i) {
        cube_ctx* c = nullptr;
        cube_status st = cube_init(&ds[i], nullptr, e->streams[i % e->sched.streams], &c);
        if (st != CUBE_OK) {
            delete e;
            return st;
        }
        e->boxes.push_back(c);
    }
    // tile classes: boxes whose tile FFTs are interchangeable
    int most = 0;
    for (int i = 0; i < nboxes; ++i) {
        const cube_ctx* c = e->boxes[i];
        const Geom& g = c->g;
        const int fmt = spec_fmt_of(ds[i]);
        TileClass* k = nullptr;
        for (TileClass& q : e->classes)
            if (q.F == g.F && q.T == g.T && q.b == g.b && q.f == g.f && q.r == g.r && q.a == g.a && q.npp == g.npp &&
                q.fdr == g.fdr && q.fmt == fmt && q.periodic == g.periodic)
                k = &q;
        if (!k) {
            e->classes.push_back(TileClass{g.F, g.T, g.b, g.f, g.r, g.a, g.npp, g.fdr, fmt, g.periodic});
            k = &e->classes.back();
            fine_window(g, false, &k->lo, &k->hi);
        }
        for (int t = 0; t < g.ntiles; ++t) k->items.push_back({i, t});
    }
    for (TileClass& k : e->classes) most = std::max<int>(most, (int)k.items.size());
    const int cap = o.tiles_in_flight ? o.tiles_in_flight : 256;
    e->max_tiles = std::max(1, std::min(cap, most));
    e->sched.tiles = o.tiles_in_flight ? o.tiles_in_flight : (have_cached ? cached.tiles : std::min(64, e->max_tiles));
    e->sched.tiles = std::min(e->sched.tiles, e->max_tiles);
    for (TileClass& k : e->classes) {
        const int64_t F = k.F, w = std::min<int64_t>(e->max_tiles, (int64_t)k.items.size());
        k.real_bytes = (size_t)(w * F * F * F + kFineRealPad) * sizeof(float);
        k.spec_bytes = (size_t)(w * F * F * (F / 2 + 1)) * 2 * sizeof(float);
        if (hipMalloc(reinterpret_cast<void**>(&k.real), k.real_bytes) != hipSuccess ||
            hipMalloc(&k.spec, k.spec_bytes) != hipSuccess) {
            (void)hipGetLastError();
            delete e;
            return fail(CUBE_OOM, "ensemble: fine workspace");
        }
    }
    *out = e;
    return CUBE_OK;
}

cube_status cube_ensemble_box(cube_ensemble* e, int32_t i, cube_ctx** out) {
    if (!e || !out || i < 0 || i >= (int32_t)e->boxes.size()) return fail(CUBE_INVALID, "no such box");
    cube_ctx* c = e->boxes[i];
    c->stream = e->stream_of(i);
    c->mem.stream = c->stream;
    *out = c;
    return CUBE_OK;
}

cube_status cube_ensemble_step(cube_ensemble* e, int32_t nsteps) {
    if (!e) return fail(CUBE_INVALID, "null ensemble");
    if (nsteps < 0) return fail(CUBE_INVALID, "negative step count");
    for (cube_ctx* c : e->boxes) {
        cube_status st = check_ctx(c);
        if (st != CUBE_OK) return st;
        if (c->prof.on) return fail(CUBE_INVALID, "ensemble boxes cannot be profiled");
    }
    if (hipSetDevice(e->device) != hipSuccess) return fail(CUBE_DEVICE, "bad device");
    if (!e->tuned && nsteps > 0) {
        cube_status st = tune(e, nullptr);
        if (st != CUBE_OK) return st;
    }
    return run_ensemble(e, nsteps);
}

cube_status cube_ensemble_tune(cube_ensemble* e, cube_ensemble_desc* chosen) {
    if (!e) return fail(CUBE_INVALID, "null ensemble");
    if (hipSetDevice(e->device) != hipSuccess) return fail(CUBE_DEVICE, "bad device");
    const bool as = e->auto_streams, at = e->auto_tiles;
    e->auto_streams = e->auto_tiles = true;
    cube_status st = tune(e, chosen);
    e->auto_streams = as;
    e->auto_tiles = at;
    if (chosen) chosen->use_graph = e->use_graph ? 0 : -1;
    return st;
}

cube_status cube_ensemble_schedule(cube_ensemble* e, cube_ensemble_desc* out) {
    if (!e || !out) return fail(CUBE_INVALID, "null argument");
    std::memset(out, 0, sizeof(*out));
    out->streams = e->sched.streams;
    out->tiles_in_flight = e->sched.tiles;
    out->use_graph = e->use_graph ? 0 : -1;
    out->device = e->device;
    return CUBE_OK;
}

void cube_ensemble_destroy(cube_ensemble* e) { delete e; }

}  // extern "C"
