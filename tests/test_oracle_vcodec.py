"""Pins of the oracle's cell-mean velocity codec (Eq. (3), Eq. (4); V1-V4)."""

import numpy as np
import pytest

from cube_inputs import config, zeldovich_ics
from oracle import Box, codec, pm, step, vcodec


def test_fast_atan_error_bound():
    """Eq. (4): maximum absolute error 0.0038 rad over the whole line (the
    printed bound; the quadratic's worst case is 0.00376 near |x| = 0.64 and
    its reflection near |x| = 1.55)."""
    x = np.concatenate([np.linspace(-60.0, 60.0, 2_400_001), np.geomspace(1.0, 1e9, 200_001),
                        -np.geomspace(1.0, 1e9, 200_001)])
    err = np.abs(vcodec.fast_atan(x) - np.arctan(x))
    assert err.max() <= 0.0038
    assert err.max() > 0.0037                      # the bound is attained, not loose
    assert abs(x[np.argmax(err)]) in (pytest.approx(1.551, abs=0.01), pytest.approx(0.645, abs=0.01))


def test_fast_atan_shape():
    x = np.linspace(0.0, 50.0, 100_001)
    assert np.array_equal(vcodec.fast_atan(-x), -vcodec.fast_atan(x))
    assert vcodec.fast_atan(np.array([1.0]))[0] == np.pi / 4
    assert vcodec.fast_atan(np.array([0.0]))[0] == 0.0
    # continuous at |x| = 1 and monotone
    assert np.all(np.diff(vcodec.fast_atan(x)) > 0)
    assert vcodec.fast_atan(np.array([1e12]))[0] == pytest.approx(np.pi / 2, abs=1e-11)


def test_every_code_round_trips():
    """0.0038 rad < pi / 510 (half a code's angle), so encode(decode(u)) = u."""
    u = np.arange(-127, 128)
    assert 0.0038 < np.pi / 510
    for sigma in (2.0 ** -12, 2.0 ** -3, 1.0, 64.0):
        back, sat = vcodec.encode_deviation(vcodec.decode_deviation(u, sigma), sigma)
        assert np.array_equal(back.astype(np.int64), u) and sat == 0


def test_decode_table():
    T = vcodec.deviation_table()
    assert T.size == 255 and T[127] == 0.0
    assert np.all(np.diff(T) > 0)
    assert np.allclose(T, -T[::-1], rtol=0, atol=1e-12)
    assert T[-1] == pytest.approx(np.tan(127 * np.pi / 255))


def test_round_trip_deviation_bound():
    """A deviation within the code range comes back within the angle error
    of one half code plus Eq. (4)'s error, mapped through tan."""
    rng = np.random.default_rng(5)
    sigma = 0.25
    dv = sigma * np.tan(rng.uniform(-1.55, 1.55, 200_000))
    u, sat = vcodec.encode_deviation(dv, sigma)
    assert sat == 0
    back = vcodec.decode_deviation(u, sigma)
    th = np.arctan(np.abs(dv) / sigma)
    d = np.pi / 510 + 0.0038
    bound = sigma * (np.tan(np.minimum(th + d, np.pi / 2 - 1e-9)) - np.tan(th))
    assert np.all(np.abs(back - dv) <= bound * (1 + 1e-12) + 1e-15)
    # beyond the last code's value: last code, counted as saturated
    tmax = np.tan(127 * np.pi / 255)
    big = np.array([sigma * tmax * 1.01, -sigma * 1e6, sigma * tmax * 0.999])
    u2, sat2 = vcodec.encode_deviation(big, sigma)
    assert sat2 == 2 and list(u2) == [127, -127, 127]


def test_cell_means_brute_force():
    """Sequential FP64 sums per cell, divided by the count, rounded to FP32
    (a plain loop; counts up to 40 so the summation order matters)."""
    rng = np.random.default_rng(6)
    counts = rng.integers(0, 40, 60)
    counts[:3] = 0
    v = rng.standard_normal((counts.sum(), 3)) * 10.0 ** rng.integers(-3, 3, (counts.sum(), 1))
    vc = vcodec.cell_means(counts, v)
    k = 0
    for c, n in enumerate(counts):
        acc = [0.0, 0.0, 0.0]
        for i in range(k, k + n):
            for a in range(3):
                acc[a] = acc[a] + float(v[i, a])
        want = np.array([x / n for x in acc]) if n else np.zeros(3)
        assert np.array_equal(vc[c], want.astype(np.float32))
        k += n
    assert vc.dtype == np.float32


def test_sigma_is_power_of_two_above_rms():
    rng = np.random.default_rng(7)
    dv = 0.013 * rng.standard_normal((1000, 3))
    s = vcodec.deviation_scale(dv)
    rms = np.sqrt(np.mean(dv ** 2))
    assert s >= rms > s / 2 and np.log2(s) == np.round(np.log2(s))
    assert vcodec.deviation_scale(np.zeros((4, 3))) == 1.0


def test_state_decodes_cell_mean_plus_deviation():
    box = Box.from_spec(config("t4").with_(vel_codec=1)).validate()
    spec = config("t4")
    pos, vel = zeldovich_ics(spec.n_side, spec.spectral_index, spec.rms_disp, spec.seed, spec.dt)
    st = codec.compress(box, pos, vel, with_ids=True)
    assert st.vc is not None and st.vc.shape == (box.n_cells, 3)
    v = st.velocities()
    cell = st.cell_canon()
    assert np.array_equal(v, st.vc[cell].astype(np.float64) + st.s * vcodec.deviation_table()[st.u.T.astype(np.int64) + 127])
    # each cell's mean of the stored velocities (by id) is its v_c, to FP32 rounding
    v_in = np.asarray(vel, np.float64)[st.ids]
    got = vcodec.cell_means(st.counts, v_in)
    assert np.array_equal(got, st.vc)


def test_cell_mean_codec_beats_linear_codec_on_zeldovich_velocities():
    """Same six bytes per particle: the cell-mean codec's velocity error is
    far below the linear codec's (the cell mean carries the bulk flow)."""
    spec = config("c2s")
    pos, vel = zeldovich_ics(spec.n_side, spec.spectral_index, spec.rms_disp, spec.seed, spec.dt)
    errs = {}
    for vcode in (0, 1):
        box = Box.from_spec(spec.with_(vel_codec=vcode)).validate()
        st = codec.compress(box, pos, vel, with_ids=True)
        errs[vcode] = np.sqrt(np.mean((st.velocities() - np.asarray(vel, np.float64)[st.ids]) ** 2))
    assert errs[1] < 0.25 * errs[0], errs


def test_cell_mean_step_is_exact_drift_and_stable_order():
    """One step with the cell-mean codec: the new state decodes to the FP32
    kicked velocities within the codec bound, and positions moved by exactly
    v32 (256/H) dt quanta (floor)."""
    spec = config("t4").with_(vel_codec=1)
    box = Box.from_spec(spec).validate()
    pos, vel = zeldovich_ics(spec.n_side, spec.spectral_index, spec.rms_disp, spec.seed, spec.dt)
    st = codec.compress(box, pos, vel, with_ids=True)
    sol = pm.Solver(box)
    new, info = step.step(sol, st, workers=1, return_info=True)
    v32 = step.kick_cell_mean(box, st, info["acc"])
    Q_old = np.empty_like(st.quanta())
    Q_old[st.ids] = st.quanta()
    Q_new = np.empty_like(Q_old)
    Q_new[new.ids] = new.quanta()
    v_by_id = np.empty_like(v32)
    v_by_id[st.ids] = v32
    X = Q_old.astype(np.float64) + 0.5 + v_by_id.astype(np.float64) * (256.0 / box.H) * box.dt
    L = 256 * box.n_coarse
    assert np.array_equal(np.mod(np.floor(X).astype(np.int64), L), Q_new)
    # re-encoded against the new cells: decode error within the codec bound
    vd = np.empty((st.n, 3))
    vd[new.ids] = new.velocities()
    dv = np.abs(vd - v_by_id)
    assert np.max(dv) <= new.s * np.tan(np.pi / 510 + 0.0038) * 200     # well inside the range
    assert np.sqrt(np.mean(dv ** 2)) < 0.01 * np.sqrt(np.mean(v_by_id.astype(np.float64) ** 2))
    assert new.saturations == 0
