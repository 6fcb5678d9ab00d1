"""Pins of the oracle's extended PP force (Sec. II optional PP module;
readings P1-P4)."""

import math

import numpy as np
import pytest
from scipy import integrate

from cube_inputs import config
from oracle import Box, cic, codec, ewald, float_mode, green, pm, pp


def _s2_force_fourier(r, D):
    """Attraction of two S2 clouds from the radial transform of the potential
    -S(k D/2)^2 / k^2: F = I / (2 pi^2 r^2) - I' / (2 pi^2 r) with
    I = int S^2 sin(kr)/k dk and I' = int S^2 cos(kr) dk."""
    S2 = lambda k: float(green.s2_window(np.array([k * D / 2.0]))[0]) ** 2
    k0 = 40.0 / D
    I = integrate.quad(lambda k: S2(k) * r * np.sinc(k * r / np.pi), 0.0, k0, limit=400, epsabs=1e-14)[0] \
        + integrate.quad(lambda k: S2(k) / k, k0, np.inf, weight="sin", wvar=r, limlst=200)[0]
    Ip = integrate.quad(lambda k: S2(k) * np.cos(k * r), 0.0, k0, limit=400, epsabs=1e-14)[0] \
        + integrate.quad(S2, k0, np.inf, weight="cos", wvar=r, limlst=200)[0]
    return I / (2 * math.pi ** 2 * r * r) - Ip / (2 * math.pi ** 2 * r)


@pytest.mark.parametrize("D", [1.0, 2.5])
def test_s2_pair_force_is_the_transform_of_the_split(D):
    """P3's polynomial against the numerical transform of S^2 / k^2, in both
    branches and beyond the diameter."""
    r = np.array([0.04, 0.17, 0.31, 0.5, 0.66, 0.83, 0.97, 1.3]) * D
    want = np.array([_s2_force_fourier(x, D) for x in r])
    assert np.allclose(pp.s2_pair_force(r, D), want, rtol=2e-7, atol=0)


def test_s2_pair_force_joins_continuously_and_turns_newtonian():
    D = 1.7
    eps = 1e-9
    for xi in (1.0, 2.0):
        r = xi * D / 2
        lo, hi = pp.s2_pair_force(np.array([r - eps, r + eps]), D)
        assert abs(lo - hi) < 1e-7 * hi
    r = np.array([1.0, 1.5, 4.0]) * D
    assert np.allclose(pp.s2_pair_force(r, D), 1.0 / (4 * np.pi * r * r), rtol=1e-14)
    # small r: the clouds' attraction grows linearly (no singularity)
    r = np.array([1e-6, 2e-6]) * D
    f = pp.s2_pair_force(r, D)
    assert f[1] == pytest.approx(2 * f[0], rel=1e-6)


def test_pair_force_support():
    r_pp = 2.0
    r = np.array([0.0, 1e-3, 0.5, 1.999, 2.0, 2.5])
    f = pp.pair_force(r, r_pp)
    assert f[0] == 0.0 and f[4] == 0.0 and f[5] == 0.0
    assert np.all(f[1:4] > 0)
    # Newton's 1/(4 pi r^2) dominates as r -> 0
    assert f[1] * 4 * np.pi * 1e-6 == pytest.approx(1.0, rel=1e-5)
    assert f[3] < 1e-6 * 1.0 / (4 * np.pi * 1.999 ** 2)


def _clustered_box(seed, npp):
    spec = config("c1").with_(n_side=16, pp_range=npp)
    box = Box.from_spec(spec).validate()
    rng = np.random.default_rng(seed)
    L = float(spec.n_side)
    n = spec.n_side ** 3
    centres = rng.uniform(0, L, (n // 16, 3))
    pos = np.mod(centres[rng.integers(0, centres.shape[0], n)] + 0.6 * rng.standard_normal((n, 3)), L)
    Q = codec.encode_positions(box, pos)
    st = codec.build_state(box, Q, np.zeros((n, 3), np.int8), 1.0, 0)
    return box, st


def _brute_force(box, st):
    """All pairs, minimum image, one particle at a time."""
    Q = st.quanta()
    L = 256 * box.n_coarse
    r_pp = box.pp_range * box.h
    out = np.zeros((Q.shape[0], 3))
    for i in range(Q.shape[0]):
        dq = Q - Q[i]
        dq = (dq + L // 2) % L - L // 2
        d = dq * (box.H / 256.0)
        r = np.sqrt(np.sum(d * d, axis=1))
        near = (r > 0) & (r < r_pp)
        rn = r[near]
        f = 1.0 / (4 * np.pi * rn * rn) - pp.s2_pair_force(rn, r_pp)
        out[i] = np.sum((f / rn)[:, None] * d[near], axis=0)
    return out


@pytest.mark.parametrize("npp", [1, 4])
def test_cell_search_equals_all_pairs(npp):
    """P4: the 27-cell search finds every pair inside r_pp (wrapping the
    periodic box included)."""
    box, st = _clustered_box(11, npp)
    got = pp.pp_accel(box, st)
    want = _brute_force(box, st)
    scale = np.max(np.abs(want))
    assert scale > 0
    assert np.max(np.abs(got - want)) <= 1e-12 * scale
    # sampled evaluation from the planes gives the same values
    cells = np.array([0, 5, box.n_cells // 2, box.n_cells - 1])
    idx, a = pp.pp_accel_cells(box, st.counts, st.offsets(), st.m, cells)
    assert np.max(np.abs(a - want[idx])) <= 1e-12 * scale


def test_pp_conserves_momentum():
    box, st = _clustered_box(12, 4)
    a = pp.pp_accel(box, st)
    assert np.max(np.abs(a.sum(axis=0))) <= 1e-10 * np.abs(a).sum()


def test_fine_kernel_limit_and_reduction():
    """The corrected kernel at k = 0 and its reduction to the plain one."""
    h, a_len = 0.5, 6.0
    G0 = green.short_range_green_continuum(16, h, a_len)
    G1 = green.short_range_green_continuum(16, h, a_len, pp_len=2.0)
    assert G1[0, 0, 0] == pytest.approx(-(a_len ** 2 - 4.0) / 30.0)
    # the difference is the PP part -(1 - S_pp^2)/k^2
    k2 = green._k2_grid(16, h, False)
    Spp = green.s2_window(np.sqrt(k2) * 1.0)
    with np.errstate(divide="ignore", invalid="ignore"):
        want = -(1.0 - Spp ** 2) / k2
    want[0, 0, 0] = -4.0 / 30.0
    assert np.allclose(G0 - G1, want, rtol=1e-12, atol=1e-15)


def _total_force(box, src, tp, with_pp):
    fs = float_mode.FloatSolver(box)
    rho_c = cic.deposit(src / box.H, box.n_coarse) / box.H ** 3
    g_c = pm.fd_gradient(pm.solve(rho_c, fs.Gc), box.H)
    rho_f = cic.deposit(src / box.h, box.n_fine) / box.h ** 3
    g_f = pm.fd_gradient(pm.solve(rho_f, fs.Gf), box.h)
    a = cic.gather(g_f, tp / box.h).T + cic.gather(g_c, tp / box.H).T
    if with_pp:
        L = float(box.n_side)
        d = np.mod(src - tp + L / 2, L) - L / 2
        r = np.linalg.norm(d, axis=1)
        a = a + (pp.pair_force(r, box.pp_range * box.h) / r)[:, None] * d
    return a


def test_mesh_plus_pp_follows_newton_inside_the_pp_range():
    """Both meshes with the corrected fine kernel plus the pair force give a
    close pair nearly Newton's force, where the meshes alone fall far short."""
    src = np.array([[10.3, 12.7, 15.1]])
    rng = np.random.default_rng(3)
    res = {}
    for npp in (0, 4):
        box = Box.from_spec(config("c1").with_(pp_range=npp)).validate()
        for lo, hi in [(0.1, 0.3), (0.3, 0.6)]:
            r = rng.uniform(lo, hi, 300)
            dirs = rng.standard_normal((300, 3))
            dirs /= np.linalg.norm(dirs, axis=1)[:, None]
            tp = np.mod(src + dirs * r[:, None], 32.0)
            a = _total_force(box, src, tp, npp > 0)
            fe = ewald.ewald_force(np.mod(tp - src + 16.0, 32.0) - 16.0, 32.0)
            err = np.linalg.norm(a - fe, axis=1) / np.linalg.norm(fe, axis=1)
            res[npp, lo] = np.sqrt(np.mean(err ** 2))
    assert res[4, 0.1] < 0.02 and res[4, 0.3] < 0.08
    assert res[0, 0.1] > 0.8 and res[0, 0.3] > 0.5


def test_box_validation():
    Box.from_spec(config("c1").with_(pp_range=4)).validate()
    with pytest.raises(AssertionError):
        Box.from_spec(config("c1").with_(pp_range=5)).validate()      # beyond one coarse cell
    Box.from_spec(config("c2s").with_(pp_range=8)).validate()
