"""Comoving integration in an expanding background (the paper's application
runs a LambdaCDM box from redshift 99 to 0, Sec. IV; its integrator is not
spelled out there).

Test infrastructure: part of the FP64 oracle.

Readings (C1-C4):

* C1  variables: comoving positions x in mean spacings, time variable the
      scale factor a, canonical momentum p = a^2 dx/dt with time in units of
      1/H0; the state's velocity codes store p.
* C2  equations: dx/dt = p / a^2 and dp/dt = -grad phi with
      lap phi = (3/2) Omega_m delta / a; the PM solver gives phi_1 with
      lap phi_1 = delta (R1), so phi = (3/2) Omega_m phi_1 / a.
      H(a) = sqrt(Omega_m a^-3 + Omega_k a^-2 + Omega_L), Omega_k = 1 - Omega_m - Omega_L.
* C3  kick-drift leapfrog in a with a constant step da (Box.dt):
      a_n = a_start + n da; p lives at a_{n-1/2}.
        kick  p += F_1(x_n) K_n,   K_n = (3/2) Omega_m int_{a_n - da/2}^{a_n + da/2} da' / (a'^2 H(a'))
        drift x += p D_n,          D_n = int_{a_n}^{a_{n+1}} da' / (a'^3 H(a'))
      (dt = da / (a H)), with F_1 = -grad phi_1 the static-unit force.
* C4  D_n is rounded to FP32 before use, so the drift stays exact in FP64
      (R15 with D_n in place of dt); K_n stays FP64.  Integrals by 32-point
      Gauss-Legendre quadrature on each interval.

Pins (tests/test_oracle_cosmo.py): the quadrature against the closed forms
of an Einstein-de Sitter background (H = a^-3/2: K = 3 (sqrt(a2) - sqrt(a1)),
D = 2 (a1^-1/2 - a2^-1/2)) and against scipy's adaptive quadrature for
LambdaCDM; in EdS a long mode whose static-unit force is R psi grows as
psi ~ a^n with n (n + 1/2) = (3/2) R (n = 1, the linear growth factor, for
R = 1), which the leapfrog reproduces at second order in da.
"""

import numpy as np

_GL_X, _GL_W = np.polynomial.legendre.leggauss(32)


def hubble(a, omega_m: float, omega_l: float):
    omega_k = 1.0 - omega_m - omega_l
    a = np.asarray(a, dtype=np.float64)
    return np.sqrt(omega_m / a ** 3 + omega_k / a ** 2 + omega_l)


def _integrate(f, a1: float, a2: float) -> float:
    half = 0.5 * (a2 - a1)
    mid = 0.5 * (a2 + a1)
    return float(half * np.sum(_GL_W * f(mid + half * _GL_X)))


def kick_factor(a1: float, a2: float, omega_m: float, omega_l: float) -> float:
    """(3/2) Omega_m int_{a1}^{a2} da / (a^2 H(a))."""
    return 1.5 * omega_m * _integrate(lambda a: 1.0 / (a * a * hubble(a, omega_m, omega_l)), a1, a2)


def drift_factor(a1: float, a2: float, omega_m: float, omega_l: float) -> float:
    """int_{a1}^{a2} da / (a^3 H(a))."""
    return _integrate(lambda a: 1.0 / (a ** 3 * hubble(a, omega_m, omega_l)), a1, a2)


def scale_factor(box, step: int) -> float:
    return box.a_start + step * box.dt


def step_factors(box, step: int):
    """(K_n in FP64, D_n rounded to FP32 then widened) of step n (C3, C4)."""
    a = scale_factor(box, step)
    da = box.dt
    K = kick_factor(a - 0.5 * da, a + 0.5 * da, box.omega_m, box.omega_l)
    D = float(np.float32(drift_factor(a, a + da, box.omega_m, box.omega_l)))
    return K, D
