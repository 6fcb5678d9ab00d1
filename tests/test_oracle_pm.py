"""Pins of the oracle's two-level PM force (Sec. II, Eq. (1); R10-R14, R18)."""

import math

import numpy as np
import pytest
from scipy import integrate

from cube_inputs import config, zeldovich_ics
from oracle import Box, cic, codec, ewald, float_mode, green, pm


def box_of(name):
    return Box.from_spec(config(name)).validate()


def test_fd_gradient_closed_form():
    n, h, m = 16, 0.5, 3
    i = np.arange(n)
    k = 2 * np.pi * m / (n * h)
    phi = np.sin(k * i * h)[:, None, None] * np.ones((n, n, n))
    g = pm.fd_gradient(phi, h)
    expect = -np.cos(k * i * h) * np.sin(k * h) / h
    assert np.max(np.abs(g[0] - expect[:, None, None])) < 1e-14
    assert np.max(np.abs(g[1])) < 1e-15 and np.max(np.abs(g[2])) < 1e-15


def test_fd4_gradient_closed_form():
    """4-point central difference of a sine wave: the derivative's Fourier
    factor is (8 sin(kh) - sin(2kh)) / (6h), exactly."""
    n, h, m = 16, 0.5, 3
    i = np.arange(n)
    k = 2 * np.pi * m / (n * h)
    phi = np.sin(k * i * h)[None, None, :] * np.ones((n, n, n))
    g = pm.fd_gradient(phi, h, order=4)
    expect = -np.cos(k * i * h) * (8 * np.sin(k * h) - np.sin(2 * k * h)) / (6 * h)
    assert np.max(np.abs(g[2] - expect[None, None, :])) < 1e-14
    assert np.max(np.abs(g[0])) < 1e-15 and np.max(np.abs(g[1])) < 1e-15


def test_fd_orders_converge_at_their_order():
    """Halving the cell of a resolved wave cuts the 2-point error by 4 and
    the 4-point error by 16 (leading terms (kh)^2/6 and (kh)^4/30)."""
    def err(n, order):
        h = 1.0 / n
        x = (np.arange(n) + 0.5) * h
        k = 2 * np.pi
        phi = np.cos(k * x)[:, None, None] * np.ones((n, 2, 2))
        g = pm.fd_gradient(phi, h, order=order)[0][:, 0, 0]
        return np.max(np.abs(g - k * np.sin(k * x))) / k
    for order, ratio, lead in ((2, 4.0, lambda kh: kh ** 2 / 6), (4, 16.0, lambda kh: kh ** 4 / 30)):
        e1, e2 = err(64, order), err(128, order)
        assert abs(e1 / e2 - ratio) < 0.01 * ratio
        assert abs(e2 / lead(2 * np.pi / 128) - 1) < 0.01
    with pytest.raises(ValueError):
        pm.fd_gradient(np.zeros((4, 4, 4)), 1.0, order=3)


@pytest.mark.parametrize("order", [2, 4])
def test_potential_plus_difference_equals_eq1_kernel(order):
    """Eq. (1): F^i = IDFT(rho_hat K^i).  The potential-plus-difference route
    is Eq. (1) with K^i(k) = -i sin(k_i h)/h * G(k) for 2-point differences and
    -i (8 sin(k_i h) - sin(2 k_i h))/(6h) * G(k) for 4-point ones."""
    box = box_of("c1")
    rng = np.random.default_rng(0)
    n, h = box.n_coarse, box.H
    rho = rng.standard_normal((n, n, n))
    G = green.coarse_green(box)
    g = pm.fd_gradient(pm.solve(rho, G), h, order)
    modes = np.fft.fftfreq(n, d=1.0 / n)
    kx = 2 * np.pi * modes / (n * h)
    kz = 2 * np.pi * np.fft.rfftfreq(n, d=1.0 / n) / (n * h)
    ks = [kx[:, None, None], kx[None, :, None], kz[None, None, :]]
    rk = np.fft.rfftn(rho)
    for ax in range(3):
        kh = ks[ax] * h
        D = np.sin(kh) / h if order == 2 else (8 * np.sin(kh) - np.sin(2 * kh)) / (6 * h)
        K = -1j * D * G
        F = np.fft.irfftn(rk * K, s=(n, n, n), axes=(0, 1, 2))
        assert np.max(np.abs(F - g[ax])) < 1e-13 * np.max(np.abs(g[ax]))


def _state_from_positions(box, pos):
    pos = np.asarray(pos, dtype=np.float64)
    return codec.compress(box, pos, np.zeros_like(pos), with_ids=True)


@pytest.mark.parametrize("name,order", [("c1", 2), ("t4", 2), ("c1", 4), ("t4", 4)])
def test_pair_forces_are_antisymmetric(name, order):
    box = Box.from_spec(config(name).with_(fd_order=order)).validate()
    sol = pm.Solver(box)
    # in t4 the pair straddles a tile face (tile side 16 spacings)
    pos = [[15.3, 9.7, 20.2], [17.1, 8.9, 21.4]] if name == "t4" else \
        [[3.3, 9.7, 20.2], [5.1, 8.9, 21.4]]
    st = _state_from_positions(box, pos)
    a = sol.forces(st)
    scale = np.max(np.abs(a))
    assert scale > 1e-3
    assert np.max(np.abs(a[0] + a[1])) < 1e-13 * scale
    # the pull points from each particle to the other
    x = st.positions()
    assert np.dot(a[0], x[1] - x[0]) > 0


def test_single_particle_has_no_self_force():
    for name in ("c1", "t4"):
        box = box_of(name)
        st = _state_from_positions(box, [[7.77, 15.9, 1.03]])
        a = pm.Solver(box).forces(st)
        assert np.max(np.abs(a)) < 1e-14


@pytest.mark.parametrize("name", ["c1", "t4"])
def test_random_set_conserves_momentum(name):
    box = box_of(name)
    spec = config(name)
    pos, vel = zeldovich_ics(spec.n_side, spec.spectral_index, spec.rms_disp, spec.seed, spec.dt)
    st = codec.compress(box, pos, vel)
    a = pm.Solver(box).forces(st)
    assert np.linalg.norm(a.sum(axis=0)) <= 1e-12 * np.abs(a).sum()


@pytest.mark.parametrize("name", ["c1", "t4"])
def test_uniform_lattice_feels_no_force(name):
    box = box_of(name)
    n = box.n_side
    i = np.arange(n) + 0.5
    z, y, x = np.meshgrid(i, i, i, indexing="ij")
    st = _state_from_positions(box, np.stack([x.ravel(), y.ravel(), z.ravel()], 1))
    a = pm.Solver(box).forces(st)
    assert np.max(np.abs(a)) < 1e-12


@pytest.mark.parametrize("order", [2, 4])
def test_tiling_invariance(order):
    """R11: with a <= b - 2 - order/2 the tiled short-range force equals the
    fine force of one periodic mesh carrying the same truncated kernel."""
    spec = config("t4").with_(fd_order=order)
    box = Box.from_spec(spec).validate()
    pos, vel = zeldovich_ics(spec.n_side, spec.spectral_index, spec.rms_disp, spec.seed, spec.dt)
    st = codec.compress(box, pos, vel)
    _, a_f, a_c = pm.Solver(box).forces(st, parts=True)
    fsol = float_mode.FloatSolver(box)
    bf, bc = fsol.parts(st.positions())
    assert np.max(np.abs(a_f - bf)) < 1e-12 * np.max(np.abs(bf))
    assert np.max(np.abs(a_c - bc)) < 1e-12 * np.max(np.abs(bc))


def test_fd4_buffer_bound_is_tight():
    """With 4-point gradients one more buffer cell is needed: at a = b - 3
    the tiled fine force no longer equals the single-mesh one, and the
    geometry check refuses that box."""
    spec = config("t4").with_(fd_order=4, r_cut_fine=config("t4").buffer_fine - 3)
    box = Box.from_spec(spec)
    with pytest.raises(AssertionError):
        box.validate()
    Box.from_spec(spec.with_(fd_order=2)).validate()
    pos, vel = zeldovich_ics(spec.n_side, spec.spectral_index, spec.rms_disp, spec.seed, spec.dt)
    st = codec.compress(box, pos, vel)
    a_f, _ = pm._fine_all(box, st.quanta(), st.counts, st.offsets(), green.fine_green(box), False, 1)
    bf, _ = float_mode.FloatSolver(box).parts(st.positions())
    assert np.max(np.abs(a_f - bf)) > 1e-7 * np.max(np.abs(bf))


def _single_source_field(box, src):
    fs = float_mode.FloatSolver(box)
    rho_c = cic.deposit(src / box.H, box.n_coarse) / box.H ** 3
    g_c = pm.fd_gradient(pm.solve(rho_c, fs.Gc), box.H)
    rho_f = cic.deposit(src / box.h, box.n_fine) / box.h ** 3
    g_f = pm.fd_gradient(pm.solve(rho_f, fs.Gf), box.h)
    return g_f, g_c


def _probe(box, src, r, rng, npts):
    L = float(box.n_side)
    dirs = rng.standard_normal((npts, 3))
    dirs /= np.linalg.norm(dirs, axis=1)[:, None]
    tp = np.mod(src + dirs * np.asarray(r)[..., None], L)
    return dirs, tp


def test_far_field_matches_ewald():
    """Beyond the split radius the force is the long-range mesh force alone
    and must reproduce the periodic (Ewald) point-mass force."""
    box = box_of("c1")
    src = np.array([[10.3, 12.7, 15.1]])
    g_f, g_c = _single_source_field(box, src)
    rng = np.random.default_rng(0)
    for lo, hi, mean_tol, rms_tol in [(8.0, 12.0, 0.02, 0.05), (6.0, 8.0, 0.03, 0.08)]:
        r = rng.uniform(lo, hi, 600)
        _, tp = _probe(box, src, r, rng, 600)
        a = cic.gather(g_f, tp / box.h).T + cic.gather(g_c, tp / box.H).T
        d = np.mod(tp - src + 16.0, 32.0) - 16.0
        fe = ewald.ewald_force(d, 32.0)
        ratio = np.sum(a * fe, 1) / np.sum(fe * fe, 1)
        err = np.linalg.norm(a - fe, axis=1) / np.linalg.norm(fe, axis=1)
        assert abs(ratio.mean() - 1.0) < mean_tol
        assert np.sqrt(np.mean(err ** 2)) < rms_tol


def _analytic_short_range_force(r, a_len):
    """F_s = F_G - F_l with F_l from the radial transform of S^2/k^2."""
    def f(k):
        S = green.s2_window(np.array([k * a_len / 2]))[0]
        return S * S * (np.cos(k * r) / r - np.sin(k * r) / (k * r * r))
    v, _ = integrate.quad(f, 1e-9, 60.0, limit=4000)
    fl = -v / (2 * math.pi ** 2)
    return 1.0 / (4 * math.pi * r * r) - fl


def test_fine_mesh_force_follows_the_analytic_split():
    """The fine (short-range) mesh force of one particle follows the
    continuum F_s = F_G - F_l of the S2 split to within the fine mesh's CIC
    and difference smoothing (4% of F_G for r >= 2 fine cells)."""
    box = box_of("c1")
    src = np.array([[10.3, 12.7, 15.1]])
    g_f, _ = _single_source_field(box, src)
    rng = np.random.default_rng(1)
    a_len = box.r_cut_fine * box.h
    for r in (1.0, 2.0, 3.0, 4.0, 5.0, 6.5):
        dirs, tp = _probe(box, src, np.full(300, r), rng, 300)
        af = cic.gather(g_f, tp / box.h).T
        radial = -np.sum(af * dirs, 1).mean()
        fg = 1.0 / (4 * math.pi * r * r)
        assert abs(radial - _analytic_short_range_force(r, a_len)) < 0.04 * fg
