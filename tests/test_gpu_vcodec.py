"""GPU parity of the cell-mean velocity codec (Eq. (3) with the Eq. (4)
arctangent; vel_codec = 1) through the C ABI against the oracle's vcodec:
compression bit-exact on identical FP32 inputs, decoding to the FP32 of the
oracle's FP64 decode, and a few steps to the usual bar (positions within one
quantum for >= 99.9% of particles, by id)."""

import numpy as np
import pytest

from cube_inputs import config
from tests.gpu_common import ics, rel_l2

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _spec(name):
    return config(name).with_(vel_codec=1)


def _oracle(name):
    import oracle
    from oracle import codec
    box = oracle.Box.from_spec(_spec(name)).validate()
    pos, vel = ics(name)
    return box, codec.compress(box, pos, vel, with_ids=True)


def _gpu(name, tiles_per_batch=3):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2003_03931_amd import CubeBox
    return CubeBox(_spec(name), with_ids=True, tiles_per_batch=tiles_per_batch)


def _load(g, st):
    g.set_state(st.counts, st.m, st.u, st.s, st.M, st.ids, st.step, vc=st.vc.T)


@pytest.mark.parametrize("name", ["c1", "t4", "c2s"])
def test_vcodec_compress_is_bit_exact(name):
    box, ref = _oracle(name)
    pos, vel = ics(name)
    with _gpu(name) as g:
        g.compress(pos, vel)
        st = g.get_state()
    assert np.array_equal(st["counts"], ref.counts.astype(np.int32))
    assert np.array_equal(st["ids"], ref.ids)
    assert np.array_equal(st["m"], ref.m)
    assert np.array_equal(st["vc"], ref.vc.T)
    assert st["s"] == ref.s
    assert np.array_equal(st["u"], ref.u)
    assert st["M"] == ref.M


@pytest.mark.parametrize("name", ["t4", "c2s"])
def test_vcodec_decompress(name):
    box, ref = _oracle(name)
    with _gpu(name) as g:
        _load(g, ref)
        pos, vel = g.decompress()
    v = vel.cpu().numpy()
    want = ref.velocities().astype(np.float32)
    assert np.mean(v == want) >= 0.999
    assert np.max(np.abs(v - want)) <= 1e-6 * np.max(np.abs(want))
    assert np.array_equal(pos.cpu().numpy(), ref.positions().astype(np.float32))


@pytest.mark.parametrize("name,nsteps", [("c1", 1), ("t4", 3)])
def test_vcodec_steps_match_oracle(name, nsteps):
    from oracle import pm, step
    from tests.test_gpu_parity import _compare_by_id
    box, ref = _oracle(name)
    sol = pm.Solver(box)
    o = ref
    for _ in range(nsteps):
        o = step.step(sol, o, workers=1)
    with _gpu(name, tiles_per_batch=5) as g:
        _load(g, ref)
        g.step(nsteps)
        st = g.get_state()
        diag = g.diagnostics()
    assert st["counts"].sum() == ref.n and diag["mass"] == ref.n
    d = _compare_by_id(box, st, o)
    assert np.mean(d <= 1) >= 0.999, np.bincount(np.minimum(d, 10))
    assert np.mean(d == 0) >= 0.99
    assert st["s"] == o.s
    # decoded velocities by id against the oracle's
    from oracle import vcodec
    gv = np.empty((ref.n, 3))
    cnt = st["counts"].astype(np.int64)
    gv[st["ids"]] = vcodec.decode(cnt, st["vc"].T, st["u"].T, st["s"])
    ov = np.empty((ref.n, 3))
    ov[o.ids] = o.velocities()
    err = rel_l2(gv, ov)
    print(f"{name}: {nsteps} steps, positions within 1 quantum {np.mean(d <= 1):.6f}, velocity rel L2 {err:.2e}")
    assert err <= 1e-3


def test_vcodec_diagnostics_match_oracle():
    from oracle import diag
    box, ref = _oracle("t4")
    with _gpu("t4") as g:
        _load(g, ref)
        dg = g.diagnostics()
    mo = diag.moments(ref)
    assert dg["mass"] == mo["mass"]
    assert np.allclose(dg["momentum"], mo["momentum"], rtol=1e-9, atol=1e-9 * np.sqrt(mo["kinetic"]))
    assert dg["kinetic"] == pytest.approx(mo["kinetic"], rel=1e-9)
