"""Pins of the oracle's CIC deposit and gather (R10)."""

import itertools

import numpy as np

from oracle import cic


def dyadic_positions(rng, n, size, bits=9):
    return rng.integers(0, size * 2 ** bits, size=(n, 3)) / 2.0 ** bits


def test_total_mass_exact_periodic_and_clipped():
    rng = np.random.default_rng(1)
    X = dyadic_positions(rng, 20000, 16)
    m = cic.deposit(X, 16, periodic=True)
    assert m.sum() == 20000.0                     # exact, not approximate
    # clipped: particles at least one cell inside keep all their mass
    Xin = 1.0 + dyadic_positions(rng, 5000, 14)
    mc = cic.deposit(Xin, 16, periodic=False)
    assert mc.sum() == 5000.0


def test_particle_at_cell_centre_fills_one_cell():
    m = cic.deposit(np.array([[3.5, 7.5, 0.5]]), 8)
    assert m[3, 7, 0] == 1.0 and m.sum() == 1.0 and np.count_nonzero(m) == 1


def test_single_particle_weights_closed_form():
    X = np.array([[2.75, 5.125, 7.96875]])
    m = cic.deposit(X, 8)
    expect = np.zeros((8, 8, 8))
    for c in itertools.product((0, 1), repeat=3):
        w = 1.0
        idx = []
        for ax in range(3):
            b = X[0, ax] - 0.5
            i0 = int(np.floor(b))
            t = b - i0
            w *= t if c[ax] else 1 - t
            idx.append((i0 + c[ax]) % 8)
        expect[tuple(idx)] += w
    assert np.array_equal(m, expect)


def test_integer_shift_rolls_mesh():
    rng = np.random.default_rng(2)
    X = dyadic_positions(rng, 500, 16)
    a = cic.deposit(X, 16)
    b = cic.deposit(np.mod(X + np.array([3, 0, 5]), 16), 16)
    assert np.array_equal(np.roll(a, (3, 0, 5), axis=(0, 1, 2)), b)


def test_gather_reproduces_linear_field_exactly():
    n = 12
    i = np.arange(n) + 0.5
    f = 0.25 * i[:, None, None] - 2.0 * i[None, :, None] + 0.5 * i[None, None, :] + 1.0
    rng = np.random.default_rng(3)
    X = 1.0 + dyadic_positions(rng, 300, n - 2)
    X = np.clip(X, 0.5, n - 0.5 - 2 ** -9)
    g = cic.gather(f, X, periodic=False)
    expect = 0.25 * X[:, 0] - 2.0 * X[:, 1] + 0.5 * X[:, 2] + 1.0
    assert np.max(np.abs(g - expect)) < 1e-13


def test_deposit_gather_adjoint():
    rng = np.random.default_rng(4)
    X = dyadic_positions(rng, 400, 10)
    f = rng.standard_normal((10, 10, 10))
    lhs = float(np.sum(cic.deposit(X, 10) * f))
    rhs = float(np.sum(cic.gather(f, X)))
    assert abs(lhs - rhs) < 1e-11 * np.sum(np.abs(f))
