"""Shared fixtures of the GPU parity tests: seeded inputs, oracle states and
the HIP box handle.  Inputs come from cube_inputs; expected values come only
from the oracle."""

import numpy as np
import pytest

from cube_inputs import config, zeldovich_ics

_ICS = {}


def ics(name):
    if name not in _ICS:
        spec = config(name)
        _ICS[name] = zeldovich_ics(spec.n_side, spec.spectral_index, spec.rms_disp, spec.seed, spec.dt)
    return _ICS[name]


def oracle_state(name, with_ids=True):
    import oracle
    from oracle import codec
    spec = config(name)
    box = oracle.Box.from_spec(spec).validate()
    pos, vel = ics(name)
    return box, codec.compress(box, pos, vel, with_ids=with_ids)


def gpu_box(name, with_ids=True, tiles_per_batch=0):
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2003_03931_amd import CubeBox
    return CubeBox(config(name), with_ids=with_ids, tiles_per_batch=tiles_per_batch)


def load_state(gbox, st):
    gbox.set_state(st.counts, st.m, st.u, st.s, st.M, st.ids, st.step)


def rel_l2(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    a = a.astype(np.complex128 if np.iscomplexobj(a) else np.float64)
    b = b.astype(np.complex128 if np.iscomplexobj(b) else np.float64)
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def gpu_quanta(box, gstate):
    """Global quanta (N, 3) of a state read back from the library, in its storage order."""
    from oracle.codec import State
    gs = State(box, gstate["counts"].astype(np.int64), gstate["m"], gstate["u"], gstate["s"], gstate["M"],
               gstate["ids"])
    return gs.quanta()


def check_compaction(box, before, after):
    """The library's reordering after a step against the oracle's compaction
    (Sec. III-A cell order, R16: stable counting sort of the previous storage
    order by new canonical cell), fed with the library's own new quanta and
    codes per id so that no force rounding enters.  `before`/`after` are
    states read back from the library (ids required); bytes, ids and counts
    must be identical."""
    from oracle import codec
    n = after["ids"].size
    ids = after["ids"].astype(np.int64)
    assert np.array_equal(np.sort(ids), np.arange(n)), "ids after the step are not a permutation"
    Q_by_id = np.empty((n, 3), dtype=np.int64)
    Q_by_id[ids] = gpu_quanta(box, after)
    u_by_id = np.empty((3, n), dtype=np.int8)
    u_by_id[:, ids] = after["u"]
    old_ids = before["ids"].astype(np.int64)
    ref = codec.build_state(box, Q_by_id[old_ids], u_by_id[:, old_ids].T, after["s"], after["M"],
                            ids=old_ids.astype(np.uint32))
    assert np.array_equal(ref.counts, after["counts"].astype(np.int64)), "new counts differ"
    assert np.array_equal(ref.ids.astype(np.int64), ids), "storage order differs from the stable sort by new cell"
    assert np.array_equal(ref.m, after["m"]) and np.array_equal(ref.u, after["u"])


def compare_by_id(box, gstate, ostate):
    """Per id: periodic max |dQ| (quanta) between the library's and the
    oracle's positions, and whether all three velocity codes agree."""
    n = ostate.n
    gids = gstate["ids"].astype(np.int64)
    assert np.array_equal(np.sort(gids), np.arange(n)), "library ids are not a permutation"
    qg = np.empty((n, 3), dtype=np.int64)
    qo = np.empty_like(qg)
    qg[gids] = gpu_quanta(box, gstate)
    qo[ostate.ids] = ostate.quanta()
    L = 256 * box.n_coarse
    d = np.abs(np.mod(qg - qo + L // 2, L) - L // 2).max(axis=1)
    ug = np.empty((n, 3), dtype=np.int64)
    uo = np.empty_like(ug)
    ug[gids] = gstate["u"].T
    uo[ostate.ids] = ostate.u.T
    return d, np.all(ug == uo, axis=1)
