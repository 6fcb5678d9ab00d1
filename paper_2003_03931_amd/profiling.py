"""Turn rocprofv3 output into the short text summaries kept under profiles/.

* ``stats``: per-kernel call counts and mean durations from a
  ``rocprofv3 --kernel-trace --stats --output-format csv`` run.
* ``traffic``: HBM bytes per dispatch of every step kernel from two
  ``--pmc FETCH_SIZE`` / ``--pmc WRITE_SIZE`` runs, each counter scaled by what
  it reads for a plain device copy of known size in the same run (the bench's
  ``--calibrate-copy`` step), so the numbers are bytes, not counter units.

bench.py reads the newest traffic summary for its dominant kernel when the
summary's source digest matches the current kernels (otherwise traffic is
reported as null).

Usage:
  python -m paper_2003_03931_amd.profiling stats <kernel_stats.csv> <out.txt> <command...>
  python -m paper_2003_03931_amd.profiling traffic <fetch_dir> <write_dir> <copy_bytes> <out.txt> <command...>
"""

import csv
import glob
import hashlib
import os
import re
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
PROFILES = os.path.join(ROOT, "profiles")

# step stage (cube_profile_read name) -> kernel symbol fragment
STAGE_KERNEL = {
    "coarse_deposit": "k_coarse_deposit",
    "coarse_fft_green": "k_fft<",
    "fine_deposit": "k_deposit_zm<",
    "fine_r2c_xy": "k_r2c_plane",
    "fine_z_green": "k_zconv_half",
    "fine_c2r_xy": "k_c2r_plane",
    "gather_kick_drift": "k_gather<0,",
    "scan_counts": "k_tile_scan",
    "compact": "k_compact_brick",
    "velocity_encode": "k_vc_encode",
    "pp_force": "k_pp",
}
COPY_KERNELS = ("elementwise", "copyBuffer")


# sources whose kernels the profiled plain step never launches: the
# extended PP force (pp_range > 0), the cell-mean velocity codec
# (vel_codec = 1), the request server and the ensemble runner
NOT_IN_STEP = ("pp.hip", "vcodec.hip", "server.cpp", "ensemble.cpp")


_COMMENT = re.compile(r"//[^\n]*|/\*.*?\*/", re.S)


def _code_of(text):
    """Source text without comments and blank lines: what the compiler sees,
    so that a comment edit does not invalidate a summary."""
    lines = (ln.rstrip() for ln in _COMMENT.sub("", text).splitlines())
    return "\n".join(ln for ln in lines if ln)


def source_digest(root=None):
    """Digest of the code of the profiled step's kernels (comments ignored): a
    traffic summary is valid only for them."""
    h = hashlib.sha256()
    for f in sorted(glob.glob(os.path.join(root or HERE, "csrc", "*"))):
        if os.path.basename(f) in NOT_IN_STEP:
            continue
        with open(f, encoding="utf-8") as fh:
            h.update(os.path.basename(f).encode())
            h.update(_code_of(fh.read()).encode())
    return h.hexdigest()[:16]


def short_name(k):
    return k.replace("cube::(anonymous namespace)::", "").replace("void ", "").split("(")[0]


def stats_summary(csv_path, out_path, command):
    rows = list(csv.DictReader(open(csv_path)))
    rows.sort(key=lambda r: -float(r["TotalDurationNs"]))
    lines = [f"# rocprofv3 kernel stats", f"# command: {command}", f"# source digest: {source_digest()}",
             f"{'kernel':44s} {'calls':>7s} {'avg_us':>11s} {'total_ms':>10s} {'pct':>6s}"]
    for r in rows[:25]:
        lines.append(f"{short_name(r['Name'])[:44]:44s} {int(r['Calls']):7d} {float(r['AverageNs']) / 1e3:11.2f} "
                     f"{float(r['TotalDurationNs']) / 1e6:10.3f} {float(r['Percentage']):6.2f}")
    with open(out_path, "w") as f:
        f.write("\n".join(lines) + "\n")


def _counter_rows(d, counter):
    out = []
    for f in glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True):
        for r in csv.DictReader(open(f)):
            if r["Counter_Name"] == counter:
                out.append((int(r["Dispatch_Id"]), short_name(r["Kernel_Name"]), float(r["Counter_Value"])))
    return out


def _means(rows):
    acc = {}
    for _, k, v in rows:
        acc.setdefault(k, []).append(v)
    return {k: sum(v) / len(v) for k, v in acc.items()}


def traffic_summary(fetch_dir, write_dir, copy_bytes, out_path, command):
    frows = _counter_rows(fetch_dir, "FETCH_SIZE")
    wrows = _counter_rows(write_dir, "WRITE_SIZE")
    # the calibration dispatch: a copy-like kernel whose write count is the
    # known size and which also reads (the buffer's fill writes the same
    # size but reads nothing); the same dispatch id in the fetch run gives
    # its read count
    fetch_of = {d: v for d, _, v in frows}
    cands = [(fetch_of.get(did, 0.0), did) for did, k, v in wrows
             if any(c in k for c in COPY_KERNELS) and abs(v * 1024.0 - copy_bytes) < 0.05 * copy_bytes]
    if not cands:
        raise SystemExit("no copy kernel in the WRITE_SIZE run: run the bench with --calibrate-copy")
    _, did = max(cands)
    wv = [v for d, _, v in wrows if d == did][0]
    fv = [v for d, _, v in frows if d == did][0]
    f_scale = copy_bytes / (fv * 1024.0)
    w_scale = copy_bytes / (wv * 1024.0)
    fetch, write = _means(frows), _means(wrows)
    lines = ["# HBM traffic per dispatch from rocprofv3 --pmc FETCH_SIZE / WRITE_SIZE (KiB per dispatch),",
             f"# scaled by a {copy_bytes} B device copy in the same runs: read x{f_scale:.4f}, write x{w_scale:.4f}",
             f"# command: {command}", f"# source digest: {source_digest()}",
             f"{'kernel':40s} {'read_MB':>10s} {'write_MB':>10s} {'traffic_MB':>11s}"]
    for stage, frag in STAGE_KERNEL.items():
        ks = [k for k in fetch if frag in k]
        if not ks:
            continue
        rd = sum(fetch[k] for k in ks) / len(ks) * 1024.0 * f_scale
        wr = sum(write.get(k, 0.0) for k in ks) / len(ks) * 1024.0 * w_scale
        lines.append(f"{stage:40s} {rd / 1e6:10.3f} {wr / 1e6:10.3f} {(rd + wr) / 1e6:11.3f}")
    with open(out_path, "w") as f:
        f.write("\n".join(lines) + "\n")


def lookup_traffic(stage, workload):
    """Traffic (bytes per launch) of a stage from profiles/, or None when the
    summary is missing or was taken on different kernel sources."""
    path = os.path.join(PROFILES, f"traffic_{workload}.txt")
    if not os.path.exists(path):
        return None
    digest = None
    for line in open(path):
        if line.startswith("# source digest:"):
            digest = line.split(":", 1)[1].strip()
        elif not line.startswith("#") and line.split() and line.split()[0] == stage:
            if digest != source_digest():
                return None
            return float(line.split()[3]) * 1e6
    return None


if __name__ == "__main__":
    if sys.argv[1] == "stats":
        stats_summary(sys.argv[2], sys.argv[3], " ".join(sys.argv[4:]))
    elif sys.argv[1] == "traffic":
        traffic_summary(sys.argv[2], sys.argv[3], int(sys.argv[4]), sys.argv[5], " ".join(sys.argv[6:]))
