"""The oracle against values the paper prints (tests/golden/paper_values.txt,
each with its citation)."""

import os

import numpy as np

from cube_inputs import config, zeldovich_ics
from oracle import Box, codec, vcodec

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_values.txt")


def _golden():
    vals = {}
    for line in open(GOLDEN):
        if line.strip() and not line.startswith("#"):
            name, value = line.split()[:2]
            vals[name] = float(value)
    return vals


def test_fast_atan_error_is_the_printed_one():
    """Eq. (4)'s maximum absolute error over the real line, to the printed
    precision (four decimals)."""
    want = _golden()["fast_atan_max_abs_error_rad"]
    x = np.concatenate([np.linspace(-40.0, 40.0, 1_600_001), np.geomspace(40.0, 1e8, 100_001)])
    err = np.max(np.abs(vcodec.fast_atan(x) - np.arctan(x)))
    assert round(err, 4) == want


def test_state_takes_the_printed_bytes_per_particle():
    """Both velocity codecs store one position byte and one velocity byte per
    dimension (the cell-mean codec adds per-cell means, not per-particle
    bytes)."""
    want = _golden()["state_bytes_per_particle"]
    spec = config("c1")
    pos, vel = zeldovich_ics(spec.n_side, spec.spectral_index, spec.rms_disp, spec.seed, spec.dt)
    for vc in (0, 1):
        box = Box.from_spec(spec.with_(vel_codec=vc)).validate()
        st = codec.compress(box, pos, vel)
        per_particle = (st.m.nbytes + st.u.nbytes) / st.n
        assert per_particle == want
        assert st.m.dtype == np.uint8 and st.u.dtype == np.int8
