"""Ewald-summed periodic point-mass force (textbook reference for the force
pins; Hockney & Eastwood).

Units as the rest of the oracle (R1): lap(phi) = rho - rho_bar with 4 pi G = 1,
so an isolated unit mass pulls with 1/(4 pi r^2).  For a unit mass at the
origin of a periodic cube of side L (with its neutralising background), the
force on a test particle at displacement r is

  F(r) = - sum_n (r - nL)/(4 pi s^3) [erfc(alpha s) + 2 alpha s/sqrt(pi) e^{-alpha^2 s^2}]
         - (1/L^3) sum_{k != 0} k sin(k.r) e^{-k^2 / (4 alpha^2)} / k^2,

s = |r - nL|, k = 2 pi m / L.  Both sums are truncated where their terms fall
below 1e-15 of the leading one.

Pin: the sum is independent of the splitting parameter alpha
(tests/test_oracle_ewald.py).
"""

import math

import numpy as np
from scipy.special import erfc


def ewald_force(r, L: float, alpha: float = None, nreal: int = 3, kmax: int = 8):
    r = np.atleast_2d(np.asarray(r, dtype=np.float64))
    alpha = 2.5 / L if alpha is None else alpha
    out = np.zeros_like(r)
    # real-space images
    rng = range(-nreal, nreal + 1)
    for i in rng:
        for j in rng:
            for k in rng:
                d = r - L * np.array([i, j, k], dtype=np.float64)
                s = np.sqrt(np.sum(d * d, axis=1))
                term = erfc(alpha * s) \
                    + 2.0 * alpha * s / math.sqrt(math.pi) * np.exp(-(alpha * s) ** 2)
                with np.errstate(divide="ignore", invalid="ignore"):
                    f = -d * (term / (4.0 * math.pi * s ** 3))[:, None]
                f[s == 0.0] = 0.0
                out += f
    # reciprocal space
    m = np.arange(-kmax, kmax + 1)
    mx, my, mz = np.meshgrid(m, m, m, indexing="ij")
    kv = (2.0 * math.pi / L) * np.stack([mx.ravel(), my.ravel(), mz.ravel()], axis=1)
    k2 = np.sum(kv * kv, axis=1)
    keep = k2 > 0
    kv, k2 = kv[keep], k2[keep]
    damp = np.exp(-k2 / (4.0 * alpha * alpha)) / k2
    phase = r @ kv.T                                          # (N, K)
    out += -(np.sin(phase) * damp[None, :]) @ kv / L ** 3
    return out
