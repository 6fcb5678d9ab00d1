"""Pins of the oracle's fixed-point codec, counts and cell order (Sec. III-A,
Eq. (2); readings R4-R7, R16, R17)."""

import numpy as np
import pytest

from cube_inputs import config
from oracle import Box, codec


def box_of(name):
    return Box.from_spec(config(name)).validate()


@pytest.mark.parametrize("name", ["c1", "t4", "c2s"])
def test_position_codec_exhaustive_roundtrip(name):
    box = box_of(name)
    Q = np.arange(256 * box.n_coarse, dtype=np.int64)
    x = codec.decode_positions(box, Q)
    # decoded point is the bin centre: strictly inside the bin
    assert np.all(x > Q * box.H / 256.0) and np.all(x < (Q + 1) * box.H / 256.0)
    back = codec.encode_positions(box, np.stack([x, x, x], axis=1))
    assert np.array_equal(back[:, 0], Q) and np.array_equal(back[:, 2], Q)


@pytest.mark.parametrize("name", ["c1", "c2s"])
def test_position_codec_half_quantum_bound(name):
    box = box_of(name)
    rng = np.random.default_rng(7)
    L = float(box.n_side)
    x = rng.uniform(0.0, L, size=(100000, 3))
    y = codec.decode_positions(box, codec.encode_positions(box, x))
    d = np.abs(np.mod(y - x + L / 2, L) - L / 2)
    half_quantum = box.H / 512.0
    assert d.max() <= half_quantum
    assert d.max() > 0.99 * half_quantum            # the bound is attained, not loose


def test_position_codec_wraps_box_edge():
    box = box_of("c1")
    L = float(box.n_side)
    Q = codec.encode_positions(box, np.array([[L, -1e-9, 2 * L + 0.01]]))
    assert Q[0, 0] == 0 and Q[0, 1] == 256 * box.n_coarse - 1
    assert Q[0, 2] == codec.encode_positions(box, np.array([[0.01, 0, 0]]))[0, 0]


def test_pow2ceil_brute_force():
    rng = np.random.default_rng(3)
    xs = np.concatenate([rng.uniform(1e-6, 1e3, 2000), 2.0 ** np.arange(-20, 20),
                         2.0 ** np.arange(-20, 20) * (1 + 2 ** -52)])
    for x in xs:
        p = codec.pow2ceil(x)
        e = -60
        while 2.0 ** e < x:
            e += 1
        assert p == 2.0 ** e


def test_velocity_codec_bound_and_saturation():
    rng = np.random.default_rng(11)
    s = 2.0 ** -7
    v = rng.uniform(-127 * s, 127 * s, size=(50000, 3))
    u, sat = codec.encode_velocities(v, s)
    assert sat == 0
    assert np.max(np.abs(v - u * s)) <= s / 2
    big = np.array([[128.6 * s, -200 * s, 126.4 * s]])
    u2, sat2 = codec.encode_velocities(big, s)
    assert sat2 == 2 and list(u2[0]) == [127, -127, 126]
    # ties go to even (R17)
    u3, _ = codec.encode_velocities(np.array([[0.5 * s, 1.5 * s, -2.5 * s]]), s)
    assert list(u3[0]) == [0, 2, -2]


def test_velocity_scale_headroom():
    box = box_of("c1")
    v = np.array([[0.3, -0.1, 0.0]])
    s0 = codec.initial_velocity_scale(box, v)
    assert s0 >= 2.0 * 0.3 / 127 and s0 / 2 < 2.0 * 0.3 / 127
    assert codec.next_velocity_scale(box, s0, 0) == s0
    assert codec.next_velocity_scale(box, 1.0, 127) == 2.0      # saturated -> doubles


@pytest.mark.parametrize("name", ["t4", "c1"])
def test_canonical_order_is_a_bijection(name):
    box = box_of(name)
    c = np.arange(box.n_cells)
    cx, cy, cz = box.cell_of_canon(c)
    assert np.array_equal(box.canon(cx, cy, cz), c)
    assert cx.min() == 0 and cx.max() == box.n_coarse - 1
    # tile-major: the first Tc^3 canonical cells are exactly tile 0
    first = slice(0, box.Tc ** 3)
    assert cx[first].max() < box.Tc and cy[first].max() < box.Tc and cz[first].max() < box.Tc
    if box.tiles_per_dim == 1:
        assert np.array_equal(c, cx + box.n_coarse * (cy + box.n_coarse * cz))


def test_build_state_counts_and_stable_order_brute_force():
    box = box_of("t4")
    rng = np.random.default_rng(5)
    n = 3000
    Q = rng.integers(0, 256 * box.n_coarse, size=(n, 3))
    Q[: n // 2] = Q[0]                                      # many equal keys
    u = rng.integers(-127, 128, size=(n, 3))
    ids = np.arange(n)
    st = codec.build_state(box, Q, u, 1.0, 127, ids)
    keys = [int(box.canon(*(q // 256))) for q in Q]
    order = sorted(range(n), key=lambda i: keys[i])        # python sort is stable
    assert list(st.ids) == order
    assert st.counts.sum() == n
    for c in set(keys):
        assert st.counts[c] == keys.count(c)
    assert np.array_equal(st.quanta(), Q[order])
    assert np.array_equal(st.u.T, u[order])


def test_compress_decompress_c1():
    from cube_inputs import zeldovich_ics
    spec = config("c1")
    box = Box.from_spec(spec)
    pos, vel = zeldovich_ics(spec.n_side, spec.spectral_index, spec.rms_disp, spec.seed, spec.dt)
    st = codec.compress(box, pos, vel, with_ids=True)
    x, v = codec.decompress(st)
    L = float(box.n_side)
    d = np.abs(np.mod(x - pos[st.ids] + L / 2, L) - L / 2)
    assert d.max() <= box.H / 512.0
    assert np.max(np.abs(v - vel[st.ids])) <= st.s / 2
    assert st.M == np.max(np.abs(st.u.astype(int)))
    assert np.all(np.diff(st.cell_canon()) >= 0)
