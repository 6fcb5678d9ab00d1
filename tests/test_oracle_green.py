"""Pins of the force-split Green's functions (Sec. II; reading R12)."""

import math

import numpy as np
import pytest
from scipy import integrate

from cube_inputs import config
from oracle import Box, green


def s2_transform_numeric(k, a):
    """Fourier transform of the S2 cloud of diameter a by radial quadrature:
    rho(r) = 48/(pi a^4) (a/2 - r) for r < a/2."""
    def f(r):
        rho = 48.0 / (math.pi * a ** 4) * (a / 2 - r)
        return rho * 4.0 * math.pi * r * r * (math.sin(k * r) / (k * r) if k * r > 0 else 1.0)
    val, _ = integrate.quad(f, 0.0, a / 2, epsabs=1e-14, epsrel=1e-13, limit=200)
    return val


def test_window_at_zero_and_normalisation():
    assert green.s2_window(np.array([0.0]))[0] == 1.0
    # the cloud has unit mass
    assert abs(s2_transform_numeric(1e-9, 6.0) - 1.0) < 1e-12


@pytest.mark.parametrize("ka", [0.5, 1.9, 2.1, 3.0, 7.0, 15.0])
def test_window_matches_radial_transform(ka):
    a = 6.0
    k = ka / a
    num = s2_transform_numeric(k, a)
    ana = green.s2_window(np.array([k * a / 2.0]))[0]
    assert abs(num - ana) < 1e-10


def test_series_and_closed_form_agree_at_switch():
    xi = np.array([0.999999, 1.0, 1.000001])
    s = green.s2_window(xi)
    assert abs(s[0] - s[1]) < 1e-6 and abs(s[2] - s[1]) < 1e-6
    closed = 12.0 * (2 - 2 * np.cos(0.8) - 0.8 * np.sin(0.8)) / 0.8 ** 4
    assert abs(green.s2_window(np.array([0.8]))[0] - closed) < 1e-13


def test_short_range_limit_at_k0():
    a = 6.0
    k = 1e-3      # next series term is -(a^4/16)(1/225 + 1/280) k^2 ~ -6.5e-7
    S = green.s2_window(np.array([k * a / 2]))[0]
    assert abs((1 - S * S) / k ** 2 - a * a / 30.0) < 1e-6


@pytest.mark.parametrize("r_over_a", [1.0, 1.3, 2.0, 3.5])
def test_long_range_potential_is_newtonian_beyond_cutoff(r_over_a):
    """Sec. II: F_l(r >= r_cut) = F_G.  The long-range potential
    (1/2pi^2) int S^2 sin(kr)/(kr) dk equals the point-mass 1/(4 pi r)."""
    a = 6.0
    r = r_over_a * a

    def f(k):
        return green.s2_window(np.array([k * a / 2]))[0] ** 2 / (k * r)
    val, _ = integrate.quad(f, 1e-12, np.inf, weight="sin", wvar=r, limlst=200)
    assert abs(val / (2 * math.pi ** 2) - 1.0 / (4 * math.pi * r)) < 1e-9 / r


def test_long_range_potential_is_softened_inside_cutoff():
    a = 6.0
    r = 0.5 * a

    def f(k):
        return green.s2_window(np.array([k * a / 2]))[0] ** 2 / (k * r)
    val, _ = integrate.quad(f, 1e-12, np.inf, weight="sin", wvar=r, limlst=200)
    assert val / (2 * math.pi ** 2) < 0.97 / (4 * math.pi * r)


def test_split_sums_to_newton():
    box = Box.from_spec(config("c1"))
    n = box.n_coarse
    Gs = green.short_range_green_continuum(n, box.H, box.r_cut_fine * box.h, half_last=True)
    Gc = green.coarse_green(box)
    k2 = green._k2_grid(n, box.H, True)
    sel = k2 > 0
    assert np.max(np.abs((Gs + Gc)[sel] * k2[sel] + 1.0)) < 1e-12


@pytest.mark.parametrize("name", ["c1", "t4"])
def test_fine_kernel_even_and_truncated(name):
    box = Box.from_spec(config(name))
    K = green.fine_kernel(box)
    F = box.F
    a = box.r_cut_fine
    idx = np.arange(F)
    neg = (-idx) % F
    assert np.max(np.abs(K - K[neg][:, neg][:, :, neg])) < 1e-15 * np.max(np.abs(K))
    d = np.fft.fftfreq(F, d=1.0 / F)
    d2 = d[:, None, None] ** 2 + d[None, :, None] ** 2 + d[None, None, :] ** 2
    assert np.all(K[d2 > a * a] == 0.0)
    assert np.count_nonzero(K[d2 <= a * a]) == np.count_nonzero(d2 <= a * a)
    G = green.fine_green(box)
    assert G.shape == (F, F, F // 2 + 1)


def test_truncation_removes_only_a_small_tail():
    """The spectral short-range kernel is already concentrated inside a: the
    part cut away is a small fraction of it (a wrong window width would put a
    large share outside the sphere)."""
    box = Box.from_spec(config("c1"))
    F = box.F
    a = box.r_cut_fine
    Gs = green.short_range_green_continuum(F, box.h, a * box.h)
    K = np.fft.ifftn(Gs).real
    d = np.fft.fftfreq(F, d=1.0 / F)
    d2 = d[:, None, None] ** 2 + d[None, :, None] ** 2 + d[None, None, :] ** 2
    inside = np.sum(np.abs(K[d2 <= a * a]))
    outside = np.sum(np.abs(K[d2 > a * a]))
    assert outside < 0.05 * inside
