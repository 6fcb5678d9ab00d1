"""Pins of the oracle's kick, drift and compaction (R6-R8, R15-R17) and of the
Ewald reference."""

import numpy as np

from cube_inputs import config, zeldovich_ics
from oracle import Box, codec, ewald, pm, step


def box_of(name):
    return Box.from_spec(config(name)).validate()


def test_drift_moves_by_the_exact_displacement_and_carries():
    box = box_of("t4")
    rng = np.random.default_rng(3)
    n = 4000
    Q = rng.integers(0, 256 * box.n_coarse, size=(n, 3))
    u = rng.integers(-127, 128, size=(n, 3))
    st = codec.build_state(box, Q, u, 2.0 ** -3, 127, np.arange(n))
    s_new = codec.next_velocity_scale(box, st.s, st.M)
    u_new = st.u.T.astype(np.int64)
    Qn, carry = step.drift(box, st, u_new, s_new)
    # the displacement in quanta, from float64 global coordinates (exact here)
    D = u_new * s_new * box.dt * 256.0 / box.H
    old = st.quanta().astype(np.float64) + 0.5
    expect = np.floor(old + D).astype(np.int64) % (256 * box.n_coarse)
    assert np.array_equal(Qn, expect)
    assert np.abs(carry).max() >= 1                 # some particles change cell


def test_general_carry_beyond_one_cell():
    box = box_of("c1")
    # one particle moving 3.4 coarse cells in one step
    st = codec.build_state(box, np.array([[256 * 5 + 10, 300, 7]]), np.array([[127, 0, -127]]),
                           1.0, 127, np.array([0]))
    Qn, carry = step.drift(box, st, st.u.T.astype(np.int64), 1.0)
    assert carry[0, 0] == int(np.floor((10 + 0.5 + 127 * 128 * box.dt) / 256))
    assert carry[0, 0] >= 3 and carry[0, 2] <= -3


def test_compaction_is_a_stable_counting_sort():
    box = box_of("t4")
    spec = config("t4")
    pos, vel = zeldovich_ics(spec.n_side, spec.spectral_index, spec.rms_disp, spec.seed, spec.dt)
    st = codec.compress(box, pos, vel, with_ids=True)
    new, info = step.step(pm.Solver(box), st, return_info=True)
    # brute force: stable sort of the old order by new canonical cell
    u_new, s_new, M_new, _ = step.kick(box, st, info["acc"])
    Qn, _ = step.drift(box, st, u_new, s_new)
    keys = box.canon(*(Qn // 256).T)
    order = sorted(range(st.n), key=lambda i: keys[i])
    assert np.array_equal(new.ids, st.ids[order])
    assert np.array_equal(new.quanta(), Qn[order])
    assert new.counts.sum() == st.n
    assert np.array_equal(new.counts, np.bincount(keys, minlength=box.n_cells))
    assert new.M == np.max(np.abs(u_new)) and new.s == s_new


def test_kick_requantises_with_ties_to_even():
    box = box_of("c1")
    st = codec.build_state(box, np.array([[10, 20, 30]] * 3), np.array([[3, -5, 0]] * 3),
                           2.0 ** -4, 127, np.arange(3))
    # s' = pow2ceil(2 * 127 * s / 127) = 2 s; (u s + a dt) / s' lands on halves
    s_new = codec.next_velocity_scale(box, st.s, st.M)
    assert s_new == 2.0 ** -3
    acc = np.zeros((3, 3))
    u_new, s2, M2, sat = step.kick(box, st, acc)
    assert s2 == s_new and list(u_new[0]) == [2, -2, 0] and sat == 0   # 1.5 -> 2, -2.5 -> -2


def test_ewald_is_independent_of_alpha():
    r = np.array([[1.3, -2.2, 0.4], [7.9, 3.3, -11.0], [0.2, 0.1, 0.05]])
    f1 = ewald.ewald_force(r, 32.0, alpha=2.5 / 32, nreal=3, kmax=8)
    f2 = ewald.ewald_force(r, 32.0, alpha=4.0 / 32, nreal=2, kmax=12)
    assert np.max(np.abs(f1 - f2)) < 1e-10 * np.max(np.abs(f1))
    # close to the source the periodic force is Newtonian
    near = f1[2]
    rr = np.linalg.norm(r[2])
    assert abs(np.linalg.norm(near) * 4 * np.pi * rr ** 2 - 1.0) < 1e-3
