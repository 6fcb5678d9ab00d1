"""Ten steps of the 256^3 box with 4^3 tiles and r = 8 (the C2 geometry)
against the oracle, compared by particle id: every particle's position
within one quantum of the oracle's for >= 99.9% of the ids.

This file is collected first so that the oracle's fork-based tile workers
start before this process has initialised the GPU; if the GPU is already
initialised (the file is run after others), the oracle runs on one worker.
"""

import os

import numpy as np
import pytest

from cube_inputs import config
from tests.gpu_common import ics, load_state, oracle_state

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def test_c2_ten_steps_by_id():
    from oracle import pm, step
    name, nsteps = "c2", 10
    box, ref = oracle_state(name)
    workers = 1 if torch.cuda.is_initialized() else min(16, os.cpu_count() or 1)
    sol = pm.Solver(box)
    o = ref
    for i in range(nsteps):
        o = step.step(sol, o, workers=workers)
        print(f"oracle step {i + 1}/{nsteps} done", flush=True)
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2003_03931_amd import CubeBox
    from tests.test_gpu_parity import _compare_by_id
    with CubeBox(config(name), with_ids=True) as g:
        load_state(g, ref)
        g.step(nsteps)
        st = g.get_state()
    assert st["s"] == o.s and st["counts"].sum() == ref.n
    d = _compare_by_id(box, st, o)
    print(f"C2 {nsteps} steps: within 1 quantum {np.mean(d <= 1):.6f}, identical {np.mean(d == 0):.6f}, "
          f"max {d.max()} ({workers} oracle workers)")
    assert np.mean(d <= 1) >= 0.999
