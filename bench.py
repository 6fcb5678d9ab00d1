#!/usr/bin/env python3
"""Benchmark of the PMPM step on one MI355X.

Workload (default): the 1024^3-particle box -- 16^3 tiles of 64^3 particles,
160^3 fine FFT box per tile (128 + 2 x 16 buffer), coarse mesh 512^3, split
radius 12 fine cells, seeded Zel'dovich ICs with P(k) ~ k^-1.5 at rms
displacement 2 spacings, 6 bytes per particle, FP32 meshes.  A step is one
full cube_pm_step (deposits, both Poisson solves, gather, kick, drift,
recount, compaction) with the state resident in HBM.

Prints one JSON line: throughput in particle-steps/s, the dominant kernel's
achieved bandwidth against the 8 TB/s HBM peak (HIP events on the library
stream over the timed region), and the FP64 oracle timed on the host cores on
a bounded sample of the same tile geometry.
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


def cpu_baseline(sample="c3cpu"):
    """The FP64 oracle's step on a 256^3 box with the benchmark's tile
    geometry, tile-parallel over the host cores (run before the GPU is
    touched, so the worker processes fork from a clean process)."""
    import numpy as np
    from cube_inputs import config, zeldovich_ics
    import oracle
    from oracle import codec, pm, step

    spec = config(sample)
    box = oracle.Box.from_spec(spec).validate()
    pos, vel = zeldovich_ics(spec.n_side, spec.spectral_index, spec.rms_disp, spec.seed, spec.dt)
    st = codec.compress(box, pos, vel)
    del pos, vel
    workers = max(1, min(16, os.cpu_count() or 1))
    sol = pm.Solver(box)
    t0 = time.perf_counter()
    step.step(sol, st, workers=workers)
    dt = time.perf_counter() - t0
    n = spec.n_side ** 3
    return {"value": n / dt, "unit": "particle-steps/s", "cores": workers, "kind": "oracle",
            "sample": f"one full oracle step (coarse mesh, all {box.n_tiles} tiles, kick, drift, compaction) "
                      f"of a {spec.n_side}^3 box with the same tile geometry (r=4, b=16, 160^3 tile box, "
                      f"8 particles per coarse cell): {n} particle-steps in {dt:.2f} s"}


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
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; multi-GPU sharding is a design note only",
                          "n_gpus": args.gpus}))
        sys.exit(2)

    base = None
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle) ...")
        base = cpu_baseline()
        log(f"cpu baseline {base['value']:.3e} particle-steps/s on {base['cores']} cores")

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
    box = CubeBox(spec, tiles_per_batch=args.tiles_per_batch)
    box.compress(pos, vel)
    del pos, vel
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
    box.close()
    log(f"timed {args.steps} steps in {elapsed:.3f} s")

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
                        f"fine FFT box {box.F}^3 per tile, coarse mesh {box.n_coarse}^3, r_cut "
                        f"{spec.r_cut_fine} fine cells, Zel'dovich ICs P(k)~k^{spec.spectral_index} rms "
                        f"{spec.rms_disp}, 6 B/particle state, FP32 meshes",
            "n_particles": n,
            "precision": "fp32",
            "tiles_per_batch": args.tiles_per_batch or "auto",
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
        "cpu_baseline": base,
        "diagnostics": {"mass": diag["mass"], "max_carry": diag["max_carry"], "max_u": diag["max_u"],
                        "saturations": diag["saturations"]},
        "stages_ms_per_step": {s["name"]: s["total_ms"] / args.steps for s in stages if s["launches"]},
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
