"""GPU: a multi-step call enqueues every step without host synchronisation
and takes its decisions on the device; the host-side recovery of each halt
(sorted general compaction, FP16 range overflow, re-plan) must give exactly
the bytes of the uninterrupted path.  Conditions are forced from the host
through cube_debug_force, so every kernel runs normally."""

import numpy as np
import pytest

from tests.gpu_common import check_compaction, gpu_box, load_state, oracle_state

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _run(name, nsteps, force=None, split=False, precision="fp32"):
    from cube_inputs import config
    from paper_2003_03931_amd import CubeBox
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    box, ref = oracle_state(name)
    with CubeBox(config(name), with_ids=True, tiles_per_batch=5, precision=precision) as g:
        load_state(g, ref)
        if force:
            g.debug_force(*force)
        if split:
            for _ in range(nsteps):
                g.step(1)
        else:
            g.step(nsteps)
        st = g.get_state()
        d = g.diagnostics()
    return box, ref, st, d


def _same(a, b):
    for k in ("counts", "m", "u", "ids"):
        assert np.array_equal(a[k], b[k]), k
    assert a["s"] == b["s"] and a["M"] == b["M"] and a["step"] == b["step"]


def test_one_call_equals_single_steps():
    _, _, a, da = _run("t4", 3)
    _, _, b, db = _run("t4", 3, split=True)
    _same(a, b)
    assert a["step"] == 3 and da["step"] == 3
    assert da["saturations"] == db["saturations"] and da["max_carry"] == db["max_carry"]


def test_forced_general_compaction_equals_fast_path():
    """The sorted general path and the fast path are the same stable sort by
    new cell: forcing the general path in the middle step changes no byte."""
    box, ref, a, _ = _run("t4", 3)
    _, _, b, db = _run("t4", 3, force=(2, 1))
    _same(a, b)
    assert db["step"] == 3


def test_forced_general_compaction_order():
    box, ref = oracle_state("c1")
    from cube_inputs import config
    from paper_2003_03931_amd import CubeBox
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    with CubeBox(config("c1"), with_ids=True) as g:
        load_state(g, ref)
        before = g.get_state()
        g.debug_force(2, 1)
        g.step(1)
        after = g.get_state()
    check_compaction(box, before, after)


def test_forced_replan_changes_nothing():
    _, _, a, _ = _run("t4", 3)
    _, _, b, db = _run("t4", 3, force=(3, 1))
    _same(a, b)
    assert db["step"] == 3


def test_fp16_range_flag_reruns_with_fp32_spectra():
    """An FP16 context whose first step raises the range flag runs that step
    (and the rest of the call) with FP32 spectra: the FP32 context's bytes,
    and the saturation counter counts the step once."""
    _, _, a, da = _run("t4", 2, precision="fp32")
    _, _, b, db = _run("t4", 2, force=(1, 1), precision="fp16")
    _same(a, b)
    assert da["saturations"] == db["saturations"]
    _, _, c, _ = _run("t4", 2, precision="fp16")
    assert not all(np.array_equal(a[k], c[k]) for k in ("m", "u"))    # FP16 spectra really differ
