#!/usr/bin/env python3
"""Benchmark of the PMPM step on one MI355X.

Workload (default): the 1024^3-particle box -- 16^3 tiles of 64^3 particles,
160^3 fine FFT box per tile (128 + 2 x 16 buffer), coarse mesh 512^3, split
radius 12 fine cells, seeded Zel'dovich ICs with P(k) ~ k^-1.5 at rms
displacement 2 spacings, 6 bytes per particle, FP32 meshes.  A step is one
full cube_pm_step (deposits, both Poisson solves, gather, kick, drift,
recount, compaction) with the state resident in HBM.

Prints one JSON line: throughput in particle-steps/s (FP32 spectra; the
BF16 and FP16 spectrum stores, the cell-mean velocity codec and the extended
PP force on the same input beside it), the dominant
kernel's achieved bandwidth against the 8 TB/s HBM peak (HIP events on the
library stream over the timed region), the FP64 oracle timed on the host
cores on a bounded sample of the same tile geometry, and a served stream of
boxes at 4 and 40 requests per second (p50/p99 time to completion,
admission waits, aggregate particle-steps/s), and a batched ensemble of 96
boxes against the same boxes run one at a time.
"""

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "particle-steps/s at 1024^3 (plain vs mixed) and %HBM peak; serving p50/p99"
HBM_PEAK_GBS = 8000.0


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def _oracle_step_rate(name, workers):
    """Particle-steps/s of one full oracle step of workload `name` and its wall time."""
    from cube_inputs import config, zeldovich_ics
    import oracle
    from oracle import codec, pm, step

    spec = config(name)
    box = oracle.Box.from_spec(spec).validate()
    pos, vel = zeldovich_ics(spec.n_side, spec.spectral_index, spec.rms_disp, spec.seed, spec.dt)
    st = codec.compress(box, pos, vel)
    del pos, vel
    sol = pm.Solver(box)
    t0 = time.perf_counter()
    step.step(sol, st, workers=workers)
    dt = time.perf_counter() - t0
    n = spec.n_side ** 3
    return n / dt, dt, n, box.n_tiles


def cpu_baseline(sample="c3cpu", sample_one="c3s"):
    """The FP64 oracle's step on a 256^3 box with the benchmark's tile
    geometry, tile-parallel over the host cores, and on one core for a 128^3
    box with the same tile geometry (run before the GPU is touched, so the
    worker processes fork from a clean process)."""
    workers = max(1, min(16, os.cpu_count() or 1))
    v_all, t_all, n_all, nt_all = _oracle_step_rate(sample, workers)
    v_one, t_one, n_one, nt_one = _oracle_step_rate(sample_one, 1)
    geom = "r=4, b=16, 160^3 tile box, 8 particles per coarse cell"
    return {"value": v_all, "unit": "particle-steps/s", "cores": workers, "kind": "oracle",
            "sample": f"one full oracle step (coarse mesh, all {nt_all} tiles, kick, drift, compaction) "
                      f"of a 256^3 box with the same tile geometry ({geom}): {n_all} particle-steps in "
                      f"{t_all:.2f} s on {workers} worker processes",
            "one_core": {"value": v_one, "unit": "particle-steps/s", "cores": 1,
                         "sample": f"one full oracle step of a 128^3 box with the same tile geometry ({geom}, "
                                   f"{nt_one} tiles): {n_one} particle-steps in {t_one:.2f} s"},
            "cpu_count": os.cpu_count(), "cpu_model": _cpu_model(),
            "note": "unoptimised FP64 numpy reference, not the paper's tuned CPU code"}


def serving_requests(count, rng_seed=5000, rate=4.0):
    """The served stream: Poisson arrivals at `rate` per second, sides
    log-uniform over [64, 512] rounded to multiples of 64, steps uniform in
    [5, 50], P(k) ~ k^n with n uniform in [-2.5, -1], rms displacement 0.5,
    IC seed 5001 + i.  Returns (spec, steps, arrival_s) per request."""
    import numpy as np
    from cube_inputs import served_box
    rng = np.random.default_rng(rng_seed)
    out, t = [], 0.0
    for i in range(count):
        side = int(np.clip(64 * round(np.exp(rng.uniform(np.log(64), np.log(512))) / 64), 64, 512))
        steps = int(rng.integers(5, 51))
        t += rng.exponential(1.0 / rate)
        n_index = float(rng.uniform(-2.5, -1.0))
        out.append((served_box(side, n_index, rng_seed + 1 + i, f"req{i}"), steps, t))
    return out


def ensemble_boxes(count, rng_seed=4000):
    """The batched ensemble: sides drawn uniformly from {64, 96, 128, 192,
    256}, P(k) ~ k^n with n uniform in [-2.5, -1], rms displacement 0.5, IC
    seed 4001 + b."""
    import numpy as np
    from cube_inputs import served_box
    rng = np.random.default_rng(rng_seed)
    specs = []
    for b in range(count):
        side = int(rng.choice([64, 96, 128, 192, 256]))
        n_index = float(rng.uniform(-2.5, -1.0))
        specs.append(served_box(side, n_index, rng_seed + 1 + b, f"ens{b}"))
    return specs


def host_ics(spec):
    """Float ICs of a served box as host arrays (generated on the GPU)."""
    from cube_inputs import zeldovich_ics_device
    p, v = zeldovich_ics_device(spec.n_side, spec.spectral_index, spec.rms_disp, spec.seed, spec.dt)
    return p.cpu().numpy(), v.cpu().numpy()


def run_server(reqs, ics, slots, budget, precision, rate_scale=1.0):
    """Submit the requests to one server at their arrival times (divided by
    rate_scale); returns per-request results and the wall time."""
    from paper_2003_03931_amd import CubeServer
    with CubeServer(budget, max_slots=slots, precision=precision) as srv:
        t0 = time.perf_counter()
        tickets = []
        for (spec, steps, at), (pos, vel) in zip(reqs, ics):
            delay = at / rate_scale - (time.perf_counter() - t0)
            if delay > 0:
                time.sleep(delay)
            tickets.append(srv.submit(spec, pos, vel, steps))
        res = [srv.wait(t) for t in tickets]
        wall = time.perf_counter() - t0
    bad = [r["message"] for r in res if r["status"] != 0]
    if bad:
        raise RuntimeError(f"served request failed: {bad[0]}")
    return res, wall


def serving_report(reqs, res, wall, slots, budget, precision, rate):
    import numpy as np
    ttc = np.array([r["done_ms"] - r["submit_ms"] for r in res])
    wait = np.array([r["start_ms"] - r["submit_ms"] for r in res])
    ps = sum(spec.n_side ** 3 * steps for spec, steps, _ in reqs)
    span_s = (max(r["done_ms"] for r in res) - min(r["submit_ms"] for r in res)) * 1e-3
    sides = sorted(spec.n_side for spec, _, _ in reqs)
    return {"requests": len(res), "slots": slots, "hbm_budget_gb": budget / 1e9, "precision": precision,
            "arrival_rate_per_s": rate,
            "p50_ms": float(np.percentile(ttc, 50)), "p99_ms": float(np.percentile(ttc, 99)),
            "admission_wait_p50_ms": float(np.percentile(wait, 50)),
            "admission_wait_p99_ms": float(np.percentile(wait, 99)),
            "queued_requests": int(np.sum(wait > 1.0)),
            "particle_steps_per_s": ps / span_s, "wall_s": wall,
            "sides": {str(k): sides.count(k) for k in sorted(set(sides))},
            "workload": f"Poisson arrivals at {rate:g}/s; sides log-uniform in [64, 512] (multiples of 64); steps "
                        "uniform in [5, 50]; Zel'dovich ICs, n uniform in [-2.5, -1], rms 0.5; ICs made before the clock"}


def run_ensemble_bench(count, steps):
    """The batched ensemble against the same boxes run one at a time."""
    import torch
    from cube_inputs import zeldovich_ics_device
    from paper_2003_03931_amd import CubeBox, CubeEnsemble
    specs = ensemble_boxes(count)
    ics = [zeldovich_ics_device(s.n_side, s.spectral_index, s.rms_disp, s.seed, s.dt) for s in specs]
    torch.cuda.synchronize()
    n_total = sum(s.n_side ** 3 for s in specs)
    with CubeEnsemble(specs) as e:
        for b, (p, v) in zip(e.boxes, ics):
            b.compress(p, v)
        t = time.perf_counter()
        e.step(1)                  # schedule (autotuner), graph capture, warm-up
        tune_s = time.perf_counter() - t
        sched = e.schedule()
        t = time.perf_counter()
        e.step(steps)
        wall_e = time.perf_counter() - t
    torch.cuda.empty_cache()
    wall_1 = 0.0
    for s, (p, v) in zip(specs, ics):
        with CubeBox(s) as b:
            b.compress(p, v)
            b.step(1)
            torch.cuda.synchronize()
            t = time.perf_counter()
            b.step(steps)
            wall_1 += time.perf_counter() - t
    del ics
    torch.cuda.empty_cache()
    ps = n_total * steps
    sides = sorted(s.n_side for s in specs)
    return {"boxes": count, "particles": n_total, "steps_per_box": steps,
            "sides": {str(k): sides.count(k) for k in sorted(set(sides))},
            "schedule": sched, "first_step_with_tuning_s": tune_s,
            "ensemble_particle_steps_per_s": ps / wall_e, "ensemble_ms_per_step": 1e3 * wall_e / steps,
            "one_at_a_time_particle_steps_per_s": ps / wall_1, "speedup": wall_1 / wall_e,
            "workload": "sides from {64,96,128,192,256}, P(k)~k^n with n uniform in [-2.5,-1], rms 0.5, FP32; "
                        "tile FFTs of all boxes of one tile geometry in shared launches, hipGraph steps"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--config", default="c3")
    ap.add_argument("--tiles-per-batch", type=int, default=0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--calibrate-copy", type=int, default=0,
                    help="bytes of a plain device copy to run first (counter calibration)")
    ap.add_argument("--mixed-steps", type=int, default=10,
                    help="timed steps of each mixed-precision run (0 skips them)")
    ap.add_argument("--vcodec-steps", type=int, default=10,
                    help="timed steps with the cell-mean velocity codec (0 skips them)")
    ap.add_argument("--pp-steps", type=int, default=5,
                    help="timed steps with the extended PP force on (0 skips them)")
    ap.add_argument("--pp-range", type=int, default=4, help="PP range in fine cells of that run")
    ap.add_argument("--serving", type=int, default=40, help="requests of the serving run (0 skips it)")
    ap.add_argument("--serving-slots", type=int, default=4)
    ap.add_argument("--batched", type=int, default=96,
                    help="boxes of the batched-ensemble run (against one box at a time); 0 skips it")
    ap.add_argument("--batched-steps", type=int, default=16)
    ap.add_argument("--allocator", default="torch", choices=["torch", "hip"],
                    help="device memory of the boxes: torch's caching allocator or the library's hipMalloc")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "the benchmark runs on one GPU; sharding over several GPUs is not implemented",
                          "n_gpus": args.gpus}))
        sys.exit(2)

    base = None
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle) ...")
        base = cpu_baseline()
        log(f"cpu baseline {base['value']:.3e} particle-steps/s on {base['cores']} cores, "
            f"{base['one_core']['value']:.3e} on one core")

    import numpy as np
    import torch
    from cube_inputs import config, zeldovich_ics
    from paper_2003_03931_amd import CubeBox
    from paper_2003_03931_amd.profiling import lookup_traffic

    if args.calibrate_copy:
        # one elementwise kernel that reads and writes exactly this many bytes
        src = torch.ones(args.calibrate_copy // 4, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        torch.mul(src, 1.0, out=dst)
        torch.cuda.synchronize()
        del src, dst
        log(f"calibration copy of {args.calibrate_copy} bytes done")
    spec = config(args.config)
    n = spec.n_side ** 3
    log(f"initial conditions {spec.n_side}^3 ...")
    t = time.perf_counter()
    pos, vel = zeldovich_ics(spec.n_side, spec.spectral_index, spec.rms_disp, spec.seed, spec.dt)
    log(f"initial conditions done in {time.perf_counter() - t:.1f} s")
    box = CubeBox(spec, tiles_per_batch=args.tiles_per_batch, allocator=args.allocator)
    box.compress(pos, vel)
    log("compressed; warmup ...")
    box.step(args.warmup)
    torch.cuda.synchronize()
    log("timed steps ...")
    box.profile(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    box.step(args.steps)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    stages = box.profile_read()
    box.profile(False)
    diag = box.diagnostics()
    F, n_coarse = box.F, box.n_coarse
    box.close()
    del box
    torch.cuda.empty_cache()
    log(f"timed {args.steps} steps in {elapsed:.3f} s")

    # the same input with the 16-bit spectrum stores
    mixed = {}
    for prec in ("bf16", "fp16") if args.mixed_steps > 0 else ():
        mb = CubeBox(spec, tiles_per_batch=args.tiles_per_batch, precision=prec, allocator=args.allocator)
        mb.compress(pos, vel)
        mb.step(1)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        mb.step(args.mixed_steps)
        torch.cuda.synchronize()
        el = time.perf_counter() - t1
        mb.close()
        del mb
        torch.cuda.empty_cache()
        mixed[prec] = {"value": n * args.mixed_steps / el, "ms_per_step": 1e3 * el / args.mixed_steps,
                       "steps": args.mixed_steps}
        log(f"{prec}: {1e3 * el / args.mixed_steps:.1f} ms/step")

    # the same input with Eq. (3)'s cell-mean velocity codec (FP32 meshes)
    vcodec = None
    if args.vcodec_steps > 0:
        vb = CubeBox(spec.with_(vel_codec=1), tiles_per_batch=args.tiles_per_batch, allocator=args.allocator)
        vb.compress(pos, vel)
        vb.step(1)
        vb.profile(True)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        vb.step(args.vcodec_steps)
        torch.cuda.synchronize()
        el = time.perf_counter() - t1
        vst = {st["name"]: st["total_ms"] / args.vcodec_steps for st in vb.profile_read() if st["launches"]}
        vdiag = vb.diagnostics()
        vb.close()
        del vb
        torch.cuda.empty_cache()
        vcodec = {"value": n * args.vcodec_steps / el, "ms_per_step": 1e3 * el / args.vcodec_steps,
                  "steps": args.vcodec_steps, "velocity_encode_ms": vst.get("velocity_encode"),
                  "compact_ms": vst.get("compact"), "gather_kick_drift_ms": vst.get("gather_kick_drift"),
                  "sigma": vdiag["s"], "saturations": vdiag["saturations"]}
        log(f"cell-mean velocity codec: {1e3 * el / args.vcodec_steps:.1f} ms/step")

    # the same input with the extended PP force (pairs within pp_range fine cells)
    ppr = None
    if args.pp_steps > 0:
        pb = CubeBox(spec.with_(pp_range=args.pp_range), tiles_per_batch=args.tiles_per_batch,
                     allocator=args.allocator)
        pb.compress(pos, vel)
        pb.step(1)
        pb.profile(True)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        pb.step(args.pp_steps)
        torch.cuda.synchronize()
        el = time.perf_counter() - t1
        pst = {st["name"]: st["total_ms"] / args.pp_steps for st in pb.profile_read() if st["launches"]}
        pdiag = pb.diagnostics()
        pb.close()
        del pb
        torch.cuda.empty_cache()
        ppr = {"pp_range": args.pp_range, "value": n * args.pp_steps / el, "ms_per_step": 1e3 * el / args.pp_steps,
               "steps": args.pp_steps, "pp_force_ms": pst.get("pp_force"),
               "saturations": pdiag["saturations"], "max_u": pdiag["max_u"]}
        log(f"extended PP (range {args.pp_range}): {1e3 * el / args.pp_steps:.1f} ms/step, "
            f"pair kernel {pst.get('pp_force', 0.0):.1f} ms")
    del pos, vel

    serving = None
    if args.serving > 0:
        log(f"serving: {args.serving} requests, ICs ...")
        reqs = serving_requests(args.serving)
        ics = [host_ics(spec) for spec, _, _ in reqs]
        torch.cuda.empty_cache()
        budget = 240 * 10 ** 9
        log("serving at 4 requests/s ...")
        res, wall = run_server(reqs, ics, args.serving_slots, budget, 2)
        serving = serving_report(reqs, res, wall, args.serving_slots, budget, "fp16", 4.0)
        log(f"serving p50 {serving['p50_ms']:.0f} ms, p99 {serving['p99_ms']:.0f} ms, "
            f"{serving['particle_steps_per_s']:.3e} particle-steps/s")
        log("serving stress: the same stream at 40 requests/s ...")
        res, wall = run_server(reqs, ics, args.serving_slots, budget, 2, rate_scale=10.0)
        serving["stress"] = serving_report(reqs, res, wall, args.serving_slots, budget, "fp16", 40.0)
        log(f"stress p50 {serving['stress']['p50_ms']:.0f} ms, p99 {serving['stress']['p99_ms']:.0f} ms, "
            f"admission wait p99 {serving['stress']['admission_wait_p99_ms']:.0f} ms")
        del reqs, ics

    batched = None
    if args.batched > 0:
        log(f"batched ensemble: {args.batched} boxes ...")
        batched = run_ensemble_bench(args.batched, args.batched_steps)
        log(f"batched: {batched['ensemble_particle_steps_per_s']:.3e} particle-steps/s, "
            f"{batched['speedup']:.2f}x over one box at a time, schedule {batched['schedule']}")

    total_stage_ms = sum(s["total_ms"] for s in stages)
    for s in sorted(stages, key=lambda s: -s["total_ms"]):
        if s["launches"]:
            gbs = s["bytes"] / (s["total_ms"] * 1e-3) / 1e9
            log(f"  {s['name']:<22} {s['total_ms'] / args.steps:8.2f} ms/step "
                f"{100 * s['total_ms'] / max(total_stage_ms, 1e-9):5.1f}%  {s['launches']:6d} launches  "
                f"{gbs:7.0f} GB/s algorithmic")
    dom = max(stages, key=lambda s: s["total_ms"])
    avg_ms = dom["total_ms"] / dom["launches"]
    bytes_per_launch = dom["bytes"] / dom["launches"]
    achieved = bytes_per_launch / (avg_ms * 1e-3) / 1e9
    value = n * args.steps / elapsed
    # whole-step HBM figures: algorithmic bytes (library profiler), measured
    # bytes (calibrated rocprofv3 counters from profiles/, when they match the
    # kernels) and the floor of the method (every fine and coarse half spectrum
    # crossing HBM four times in FP32, the 12 bytes of each particle's state
    # read and written once)
    step_s = elapsed / args.steps
    alg_gb = sum(s["bytes"] for s in stages) / args.steps / 1e9
    traffic = {s["name"]: lookup_traffic(s["name"], spec.name) for s in stages if s["launches"]}
    meas_gb = None
    if traffic and all(v is not None for v in traffic.values()):
        meas_gb = sum(traffic[s["name"]] * s["launches"] / args.steps for s in stages if s["launches"]) / 1e9
    ntiles = spec.tiles_per_dim ** 3
    floor_gb = (ntiles * 4 * 8 * F * F * (F // 2 + 1) + 4 * 8 * n_coarse ** 2 * (n_coarse // 2 + 1) + 12 * n) / 1e9
    hbm = {
        "peak_gbs": HBM_PEAK_GBS,
        "algorithmic_gb_per_step": alg_gb,
        "algorithmic_frac": alg_gb / step_s / HBM_PEAK_GBS,
        "measured_gb_per_step": meas_gb,
        "measured_frac": None if meas_gb is None else meas_gb / step_s / HBM_PEAK_GBS,
        "floor_gb_per_step": floor_gb,
        "effective_frac": floor_gb / step_s / HBM_PEAK_GBS,
    }
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "particle-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * elapsed / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": f"{spec.name}: {spec.n_side}^3 particles, {spec.tiles_per_dim}^3 tiles, "
                        f"fine FFT box {F}^3 per tile, coarse mesh {n_coarse}^3, r_cut "
                        f"{spec.r_cut_fine} fine cells, Zel'dovich ICs P(k)~k^{spec.spectral_index} rms "
                        f"{spec.rms_disp}, 6 B/particle state, FP32 meshes",
            "n_particles": n,
            "precision": "fp32",
            "tiles_per_batch": args.tiles_per_batch or "auto",
            "allocator": args.allocator,
        },
        "roofline": {
            "bound": "hbm",
            "kernel": dom["name"],
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": lookup_traffic(dom["name"], spec.name),
            "avg_launch_ms": avg_ms,
            "bytes_per_launch": bytes_per_launch,
        },
        "hbm_step": hbm,
        "cpu_baseline": base,
        "mixed": mixed,
        "vel_codec_cell_mean": vcodec,
        "extended_pp": ppr,
        "serving": serving,
        "batched": batched,
        "diagnostics": {"mass": diag["mass"], "max_carry": diag["max_carry"], "max_u": diag["max_u"],
                        "saturations": diag["saturations"]},
        "stages_ms_per_step": {s["name"]: s["total_ms"] / args.steps for s in stages if s["launches"]},
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
