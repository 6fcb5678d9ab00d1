"""GPU: cube_pm_step_noalloc, the entry point for callers that cannot
allocate, against cube_pm_step on identical states, through the C ABI.

The sorted general compaction (the step's only user of temporaries) is
forced from the host, so the fixed scratch region is really used; two calls
in a row, the second on a smaller box, reuse the region.  The call must not
go through the context's allocator."""

import ctypes

import numpy as np
import pytest

from tests.gpu_common import load_state, oracle_state

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _box(name):
    from cube_inputs import config
    from paper_2003_03931_amd import CubeBox
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return CubeBox(config(name), with_ids=True, tiles_per_batch=5)


def _steps(name, nsteps, noalloc):
    from paper_2003_03931_amd._lib import check
    _, ref = oracle_state(name)
    with _box(name) as g:
        load_state(g, ref)
        g.debug_force(2, nsteps)          # every step through the sorted compaction
        calls = g.allocator.calls
        if noalloc:
            check(g.lib.cube_pm_step_noalloc(g.ctx, ctypes.c_int32(nsteps)))
            assert g.allocator.calls == calls, "cube_pm_step_noalloc allocated"
        else:
            check(g.lib.cube_pm_step(g.ctx, ctypes.c_int32(nsteps)))
            assert g.allocator.calls > calls        # the general path's temporaries
        return g.get_state()


def _same(a, b):
    for k in ("counts", "m", "u", "ids"):
        assert np.array_equal(a[k], b[k]), k
    assert a["s"] == b["s"] and a["M"] == b["M"] and a["step"] == b["step"]


def test_noalloc_matches_allocating_step_twice():
    # first call on a 64^3 box (4^3 tiles), then a smaller 32^3 box
    for name, nsteps in (("t4", 2), ("c1", 1)):
        a = _steps(name, nsteps, noalloc=False)
        b = _steps(name, nsteps, noalloc=True)
        _same(a, b)
        assert b["step"] == nsteps


def test_noalloc_refuses_boxes_above_the_region():
    from cube_inputs import config
    from paper_2003_03931_amd import CubeBox
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    with CubeBox(config("c2")) as g:                 # 256^3 particles: 268 MB of temporaries
        st = g.lib.cube_pm_step_noalloc(g.ctx, ctypes.c_int32(1))
        assert st == 1                                # CUBE_INVALID, nothing run
        assert b"scratch" in g.lib.cube_last_error()
