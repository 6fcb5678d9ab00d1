"""GPU parity of the comoving integration (cosmo.py C1-C4; comoving = 1)
through the C ABI: a few steps in an expanding LambdaCDM background against
the oracle's, to the usual bar (positions within one quantum for >= 99.9% of
particles by id, >= 99% identical), with both velocity codecs."""

import numpy as np
import pytest

from cube_inputs import config
from tests.gpu_common import ics

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

COSMO = dict(comoving=1, omega_m=0.3, omega_l=0.7, a_start=0.05, dt=float(np.float32(0.0025)))


@pytest.mark.parametrize("name,nsteps,vel_codec", [("c1", 2, 0), ("t4", 3, 0), ("t4", 2, 1)])
def test_comoving_steps_match_oracle(name, nsteps, vel_codec):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import oracle
    from oracle import codec, pm, step
    from paper_2003_03931_amd import CubeBox
    from tests.test_gpu_parity import _compare_by_id
    spec = config(name).with_(vel_codec=vel_codec, **COSMO)
    box = oracle.Box.from_spec(spec).validate()
    pos, vel = ics(name)
    ref = codec.compress(box, pos, vel, with_ids=True)
    sol = pm.Solver(box)
    o = ref
    for _ in range(nsteps):
        o = step.step(sol, o, workers=1)
    with CubeBox(spec, with_ids=True, tiles_per_batch=3) as g:
        vc = None if ref.vc is None else ref.vc.T
        g.set_state(ref.counts, ref.m, ref.u, ref.s, ref.M, ref.ids, 0, vc=vc)
        g.step(nsteps)
        st = g.get_state()
    assert st["s"] == o.s and st["counts"].sum() == ref.n and st["step"] == nsteps
    d = _compare_by_id(box, st, o)
    print(f"{name} codec {vel_codec}: {nsteps} comoving steps, within 1 quantum {np.mean(d <= 1):.6f}, "
          f"identical {np.mean(d == 0):.6f}")
    assert np.mean(d <= 1) >= 0.999, np.bincount(np.minimum(d, 10))
    assert np.mean(d == 0) >= 0.99
    # the expansion is really applied: the drift multiplier differs from dt
    K, D = oracle.cosmo.step_factors(box, 0)
    assert abs(D / box.dt - 1) > 0.5
