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
    assert lib.cube_init(ctypes.byref(bad), None, ctypes.byref(ctx)) == 1
    assert b"power" in lib.cube_last_error()
    bad2 = BoxDesc(64, 4, 2, 4, 8, 12, 0.05, 2.0, 0, 0, 0, 0)     # a > b - 3
    assert lib.cube_init(ctypes.byref(bad2), None, ctypes.byref(ctx)) == 1
    assert lib.cube_init(None, None, ctypes.byref(ctx)) == 1
