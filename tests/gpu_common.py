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
