"""Pins of the oracle's comoving integration (C1-C4 in oracle/cosmo.py)."""

import math

import numpy as np
import pytest
from scipy import integrate

from cube_inputs import config, plane_wave_ics
from oracle import Box, cosmo, float_mode

L = 32.0


@pytest.mark.parametrize("a1,a2", [(0.01, 0.0125), (0.1, 0.2), (0.5, 1.0)])
def test_eds_factors_closed_form(a1, a2):
    """H = a^-3/2: K = 3 (sqrt a2 - sqrt a1), D = 2 (a1^-1/2 - a2^-1/2)."""
    K = cosmo.kick_factor(a1, a2, 1.0, 0.0)
    D = cosmo.drift_factor(a1, a2, 1.0, 0.0)
    assert K == pytest.approx(3.0 * (math.sqrt(a2) - math.sqrt(a1)), rel=1e-13)
    assert D == pytest.approx(2.0 * (a1 ** -0.5 - a2 ** -0.5), rel=1e-13)


@pytest.mark.parametrize("om,ol", [(0.3, 0.7), (0.258, 0.742), (0.5, 0.2)])
def test_lcdm_factors_against_adaptive_quadrature(om, ol):
    ok = 1.0 - om - ol
    H = lambda a: math.sqrt(om / a ** 3 + ok / a ** 2 + ol)
    for a1, a2 in ((0.01, 0.02), (0.3, 0.35), (0.9, 1.0)):
        kq = 1.5 * om * integrate.quad(lambda a: 1.0 / (a * a * H(a)), a1, a2, epsabs=0, epsrel=1e-13)[0]
        dq = integrate.quad(lambda a: 1.0 / (a ** 3 * H(a)), a1, a2, epsabs=0, epsrel=1e-13)[0]
        assert cosmo.kick_factor(a1, a2, om, ol) == pytest.approx(kq, rel=1e-12)
        assert cosmo.drift_factor(a1, a2, om, ol) == pytest.approx(dq, rel=1e-12)


def test_step_factors_round_the_drift_to_fp32():
    box = Box.from_spec(config("t4").with_(comoving=1, omega_m=0.3, omega_l=0.7, a_start=0.05, dt=0.0025))
    K, D = cosmo.step_factors(box, 3)
    om, ol = box.omega_m, box.omega_l
    assert (om, ol, box.a_start) == tuple(float(np.float32(v)) for v in (0.3, 0.7, 0.05))   # R9
    a = box.a_start + 3 * box.dt
    assert D == float(np.float32(cosmo.drift_factor(a, a + box.dt, om, ol)))
    assert K == cosmo.kick_factor(a - box.dt / 2, a + box.dt / 2, om, ol)


def _amplitude(q, x):
    d = np.mod(x[:, 0] - q[:, 0] + L / 2, L) - L / 2
    s = np.sin(2 * np.pi * q[:, 0] / L)
    return np.sum(d * s) / np.sum(s * s)


def _growth_run(da, a0=0.1, a1=0.2, A=0.01):
    """Long mode in EdS, started on the growing mode of the mesh response."""
    spec = config("c1").with_(comoving=1, omega_m=1.0, omega_l=0.0, a_start=a0, dt=da)
    box = Box.from_spec(spec).validate()
    fs = float_mode.FloatSolver(box)
    q, _, _ = plane_wave_ics(32, A, 0.0)
    probe = q.copy()
    probe[:, 0] += A * np.sin(2 * np.pi * q[:, 0] / L)
    R = _amplitude(q, q + fs.forces(probe)) / A
    n = (-0.5 + math.sqrt(0.25 + 6.0 * R)) / 2.0
    mode = np.sin(2 * np.pi * q[:, 0] / L)
    pos = q.copy()
    pos[:, 0] += A * mode
    ah = a0 - da / 2                                  # momentum half a step back
    p = np.zeros_like(q)
    p[:, 0] = ah * ah * n * A * (ah / a0) ** n * ah ** -1.5 * mode     # p = a^2 n psi H
    steps = int(round((a1 - a0) / da))
    x, _ = float_mode.leapfrog_comoving(fs, np.mod(pos, L), p, box, steps)
    return _amplitude(q, x) / A, (a1 / a0) ** n, R, n


def test_long_mode_follows_the_eds_growth_law():
    g, want, R, n = _growth_run(0.005)
    assert 0.93 < R < 0.97 and 0.95 < n < 0.99        # mesh response below the continuum's n = 1
    assert abs(g / want - 1) < 2e-3
    assert abs(g / 2.0 - 1) < 0.05                    # the continuum law D ~ a, within the response


def test_comoving_leapfrog_is_second_order():
    errs = [_growth_run(da)[0] - _growth_run(da)[1] for da in (0.01, 0.005, 0.0025)]
    assert 3.5 < errs[0] / errs[1] < 4.5, errs
    assert 3.5 < errs[1] / errs[2] < 4.5, errs
