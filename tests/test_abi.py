"""The C-ABI library loads and exports every symbol include/cube.h declares
(no compute calls: runs without a GPU)."""

import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "cube.h")
LIB = os.path.join(ROOT, "paper_2003_03931_amd", "libcube.so")


def declared_symbols():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(cube_[a-z0-9_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared_symbols()
    for must in ("cube_init", "cube_destroy", "cube_compress", "cube_decompress", "cube_pm_step",
                 "cube_forces", "cube_get_state", "cube_set_state", "cube_diagnostics"):
        assert must in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="libcube.so not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared_symbols() if not hasattr(lib, n)]
    assert not missing, missing


@pytest.mark.skipif(not os.path.exists(LIB), reason="libcube.so not built")
def test_binding_signatures_cover_the_header():
    from paper_2003_03931_amd import SIGNATURES
    assert set(SIGNATURES) == set(declared_symbols())


@pytest.mark.skipif(not os.path.exists(LIB), reason="libcube.so not built")
def test_invalid_descriptor_is_rejected_without_a_gpu():
    """Validation happens before any device call."""
    from paper_2003_03931_amd._lib import BoxDesc, load
    lib = load()
    ctx = ctypes.c_void_p()
    bad = BoxDesc(32, 1, 2, 3, 0, 12, 0.05, 2.0, 0, 0, 0, 0)      # r = 3 is not a power of two
    assert lib.cube_init(ctypes.byref(bad), None, None, ctypes.byref(ctx)) == 1
    assert b"power" in lib.cube_last_error()
    bad2 = BoxDesc(64, 4, 2, 4, 8, 12, 0.05, 2.0, 0, 0, 0, 0)     # a > b - 3
    assert lib.cube_init(ctypes.byref(bad2), None, None, ctypes.byref(ctx)) == 1
    assert lib.cube_init(None, None, None, ctypes.byref(ctx)) == 1
    bad3 = BoxDesc(32, 1, 2, 4, 0, 12, 0.05, 2.0, 7, 0, 0, 0)     # unknown precision
    assert lib.cube_init(ctypes.byref(bad3), None, None, ctypes.byref(ctx)) == 1
    assert b"precision" in lib.cube_last_error()
    bad4 = BoxDesc(32, 1, 2, 4, 0, 12, 0.05, 2.0, 0, 0, 0, 3)     # fd_order 3
    assert lib.cube_init(ctypes.byref(bad4), None, None, ctypes.byref(ctx)) == 1
    assert b"fd_order" in lib.cube_last_error()
    bad5 = BoxDesc(32, 1, 2, 4, 0, 12, 0.05, 2.0, 0, 0, 0, 2, 2)  # vel_codec 2
    assert lib.cube_init(ctypes.byref(bad5), None, None, ctypes.byref(ctx)) == 1
    assert b"vel_codec" in lib.cube_last_error()
    p, t = ctypes.c_int64(), ctypes.c_int64()
    for om, ol, a0, ok in ((0.3, 0.7, 0.01, True), (0.0, 0.7, 0.01, False), (0.3, 0.7, 0.0, False),
                           (0.3, -0.1, 0.5, False)):
        d = BoxDesc(32, 1, 2, 4, 0, 12, 0.001, 2.0, 0, 0, 0, 2, 0, 1, om, ol, a0)
        assert (lib.cube_footprint(ctypes.byref(d), ctypes.byref(p), ctypes.byref(t)) == 0) == ok, (om, ol, a0)
        if not ok:
            assert b"comoving" in lib.cube_last_error()


@pytest.mark.skipif(not os.path.exists(LIB), reason="libcube.so not built")
def test_four_point_gradients_need_one_more_buffer_cell():
    """a <= b - 3 suffices for 2-point gradients, 4-point ones need a <= b - 4
    (the same bound the oracle's geometry check enforces)."""
    from paper_2003_03931_amd._lib import BoxDesc, load
    lib = load()
    p, t = ctypes.c_int64(), ctypes.c_int64()
    for a, order, ok in ((13, 2, True), (13, 0, True), (13, 4, False), (12, 4, True)):
        d = BoxDesc(64, 4, 2, 4, 16, a, 0.05, 2.0, 0, 0, 0, order)
        assert (lib.cube_footprint(ctypes.byref(d), ctypes.byref(p), ctypes.byref(t)) == 0) == ok, (a, order)
        if not ok:
            assert b"buffer - 4" in lib.cube_last_error()


@pytest.mark.skipif(not os.path.exists(LIB), reason="libcube.so not built")
def test_footprint_is_host_only_and_grows_with_the_batch():
    """cube_footprint validates and sizes without touching a device."""
    from cube_inputs import config
    from paper_2003_03931_amd import footprint
    spec = config("t4")
    p1, t1 = footprint(spec, tiles_per_batch=1)
    p8, t8 = footprint(spec, tiles_per_batch=8)
    F = 64 * 2 // 4 + 2 * 16
    # each extra tile in flight holds one real mesh and one FP32 half spectrum
    per_tile = 4 * F ** 3 + 8 * F * F * (F // 2 + 1)
    assert p8 - p1 >= 7 * per_tile
    n = spec.n_side ** 3
    assert p1 >= 12 * n and t1 >= 24 * n          # planes; host staging of compress
    from paper_2003_03931_amd._lib import BoxDesc, load
    lib = load()
    bad = BoxDesc(32, 1, 2, 3, 0, 12, 0.05, 2.0, 0, 0, 0, 0)
    a, b = ctypes.c_int64(), ctypes.c_int64()
    assert lib.cube_footprint(ctypes.byref(bad), ctypes.byref(a), ctypes.byref(b)) == 1
    # the cell-mean velocity codec adds 24 B per particle of working planes,
    # 12 B per coarse cell and the table
    p_vc, _ = footprint(spec.with_(vel_codec=1), tiles_per_batch=1)
    n_cells = (64 * 2 // 4) ** 3
    assert p_vc - p1 >= 24 * n + 12 * n_cells


@pytest.mark.skipif(not os.path.exists(LIB), reason="libcube.so not built")
def test_server_rejects_bad_requests_without_a_gpu():
    """Server creation and request validation are host-side; a box whose
    footprint exceeds the whole budget is refused at submit."""
    from cube_inputs import config
    from paper_2003_03931_amd._lib import Request, ServerDesc, load
    from paper_2003_03931_amd import desc_from
    lib = load()
    srv = ctypes.c_void_p()
    assert lib.cube_server_create(ctypes.byref(ServerDesc(0, 1, -1, 0, 0)), ctypes.byref(srv)) == 1
    assert lib.cube_server_create(ctypes.byref(ServerDesc(1 << 20, 0, -1, 0, 0)), ctypes.byref(srv)) == 1
    assert lib.cube_server_create(ctypes.byref(ServerDesc(1 << 20, 1, -1, 0, 0)), ctypes.byref(srv)) == 0
    try:
        spec = config("c1")
        import numpy as np
        pos = np.zeros((spec.n_side ** 3, 3), np.float32)
        req = Request(desc_from(spec), 1, 0, pos.ctypes.data, pos.ctypes.data, spec.n_side ** 3, None)
        t = ctypes.c_uint64()
        assert lib.cube_submit(srv, ctypes.byref(req), ctypes.byref(t)) == 1     # 1 MiB budget: never fits
        assert b"budget" in lib.cube_last_error()
        req.n = 5
        assert lib.cube_submit(srv, ctypes.byref(req), ctypes.byref(t)) == 1
        from paper_2003_03931_amd._lib import Result
        r = Result()
        assert lib.cube_poll(srv, ctypes.c_uint64(12345), ctypes.byref(r)) == 1
    finally:
        lib.cube_server_destroy(srv)


@pytest.mark.skipif(not os.path.exists(LIB), reason="libcube.so not built")
def test_pp_range_validation_and_footprint():
    """pp_range in [0, coarse_ratio] and below r_cut_fine; the PP planes add
    12 bytes per particle to the persistent footprint."""
    from paper_2003_03931_amd._lib import BoxDesc, load
    lib = load()
    p, t = ctypes.c_int64(), ctypes.c_int64()
    sizes = {}
    for npp, ok in ((0, True), (1, True), (4, True), (5, False), (-1, False)):
        d = BoxDesc(32, 1, 2, 4, 0, 12, 0.05, 2.0, 0, 0, 0, 2, 0, 0, 1.0, 0.0, 1.0, npp)
        assert (lib.cube_footprint(ctypes.byref(d), ctypes.byref(p), ctypes.byref(t)) == 0) == ok, npp
        if ok:
            sizes[npp] = p.value
        else:
            assert b"pp_range" in lib.cube_last_error()
    assert sizes[1] == sizes[4] and 12 * 32 ** 3 <= sizes[1] - sizes[0] <= 12 * 32 ** 3 + 256


def test_binding_structs_match_the_header_layout(tmp_path):
    """Every ctypes mirror has the C struct's size and each of its fields the
    C offset: a small C program built with the host compiler against
    include/cube.h prints them."""
    import shutil
    import subprocess
    from paper_2003_03931_amd import _lib
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no host C compiler")
    pairs = {"cube_box_desc": _lib.BoxDesc, "cube_state_view": _lib.StateView, "cube_diag": _lib.Diag,
             "cube_stage_stat": _lib.StageStat, "cube_allocator": _lib.Allocator,
             "cube_server_desc": _lib.ServerDesc, "cube_request": _lib.Request, "cube_result": _lib.Result,
             "cube_ensemble_desc": _lib.EnsembleDesc}
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "cube.h"', "int main(void) {"]
    for cname, py in pairs.items():
        lines.append(f'    printf("{cname} sizeof %zu\\n", sizeof({cname}));')
        for fname, _ in py._fields_:
            lines.append(f'    printf("{cname} {fname} %zu\\n", offsetof({cname}, {fname}));')
    lines += ["    return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run([cc, "-std=c11", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    got = {}
    for line in out:
        if line:
            cname, field, value = line.split()
            got[cname, field] = int(value)
    for cname, py in pairs.items():
        assert got[cname, "sizeof"] == ctypes.sizeof(py), cname
        for fname, _ in py._fields_:
            assert got[cname, fname] == getattr(py, fname).offset, (cname, fname)


@pytest.mark.skipif(not os.path.exists(LIB), reason="libcube.so not built")
def test_ensemble_rejects_unsupported_boxes_without_a_gpu():
    """Ensemble validation runs before any device call: comoving boxes, the
    cell-mean codec and FP16 spectra are refused, as are bad options."""
    from cube_inputs import config
    from paper_2003_03931_amd._lib import EnsembleDesc, load
    from paper_2003_03931_amd import desc_from
    lib = load()
    h = ctypes.c_void_p()
    spec = config("c1")
    for bad in (spec.with_(comoving=1, omega_m=0.3, omega_l=0.7, a_start=0.1), spec.with_(vel_codec=1)):
        arr = (type(desc_from(spec)) * 1)(desc_from(bad))
        assert lib.cube_ensemble_create(arr, 1, None, ctypes.byref(h)) == 6      # CUBE_UNSUPPORTED
    arr = (type(desc_from(spec)) * 1)(desc_from(spec, precision=2))
    assert lib.cube_ensemble_create(arr, 1, None, ctypes.byref(h)) == 6
    assert b"FP16" in lib.cube_last_error()
    arr = (type(desc_from(spec)) * 1)(desc_from(spec))
    assert lib.cube_ensemble_create(arr, 1, ctypes.byref(EnsembleDesc(5, 0, 0, 0)), ctypes.byref(h)) == 1
    assert lib.cube_ensemble_create(arr, 0, None, ctypes.byref(h)) == 1
