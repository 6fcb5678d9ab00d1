"""Green's functions of the two-level PM force split (Sec. II).

Sec. II splits gravity as F_G = F_s + F_l with F_s = 0 beyond the cut-off and
F_l = F_G there, and computes each part as a Fourier-space product, Eq. (1).
The paper defers the split's functional form to its references; reading R12
takes the compact S2 split of Hockney & Eastwood:

    S(xi) = 12 (2 - 2 cos xi - xi sin xi) / xi^4,   xi = k a_len / 2,

the transform of the S2 cloud of diameter a_len.  Two S2 clouds attract exactly
like point masses once their centres are a_len apart, so

* coarse (long range):  G_c(k) = -S^2 / k^2  (k != 0), G_c(0) = 0;
* fine (short range):   G_s(k) = -(1 - S^2) / k^2, with limit -a_len^2/30 at
  k = 0; its real-space kernel vanishes beyond a_len in the continuum.  On a
  tile box of F cells the kernel is K_f = IDFT_F[G_s], truncated to the
  minimum-image sphere |d| <= a, and G_f = DFT_F[K_f] (real and even).
  With the extended PP force on (Box.pp_range, readings P1-P4 in pp.py) the
  fine kernel leaves out what the pair force carries:
  G_s(k) = -(S_pp^2 - S^2) / k^2, S_pp the S2 transform at diameter r_pp.

Units (R1, R14): Poisson's equation is lap(phi) = rho - 1 (4 pi G = 1), the
potential is phi = IDFT(G * DFT(rho)) with rho the density (mass per unit
volume) and k = 2 pi n / (mesh side in spacings); no CIC deconvolution.

Small xi uses the Taylor series of S (its closed form cancels badly there).

Pins (tests/test_oracle_green.py): S(0) = 1; S against a numerical radial
transform of the S2 profile; (1 - S^2)/k^2 -> a^2/30; K_f even and zero beyond
a; the split kernels sum to -1/k^2.
"""

import math

import numpy as np

from .geometry import Box

# S(xi) = sum_j c_j xi^(2j),  c_j = (-1)^j 12 (2j+2) / (2j+4)!
_S_SERIES = [(-1) ** j * 12.0 * (2 * j + 2) / math.factorial(2 * j + 4) for j in range(10)]


def s2_window(xi):
    """S2 cloud transform S(xi), vectorised, float64."""
    xi = np.asarray(xi, dtype=np.float64)
    out = np.empty_like(xi)
    small = xi < 1.0
    xs = xi[small] ** 2
    acc = np.zeros_like(xs)
    for c in reversed(_S_SERIES):
        acc = acc * xs + c
    out[small] = acc
    xl = xi[~small]
    out[~small] = 12.0 * (2.0 - 2.0 * np.cos(xl) - xl * np.sin(xl)) / xl ** 4
    return out


def _k2_grid(n: int, cell: float, half_last: bool):
    modes = np.fft.fftfreq(n, d=1.0 / n)
    kx = 2.0 * np.pi * modes / (n * cell)
    kz = 2.0 * np.pi * (np.fft.rfftfreq(n, d=1.0 / n) if half_last else modes) / (n * cell)
    return kx[:, None, None] ** 2 + kx[None, :, None] ** 2 + kz[None, None, :] ** 2


def coarse_green(box: Box) -> np.ndarray:
    """G_c on the coarse mesh in rfftn layout [kx, ky, kz(half)]."""
    a_len = box.r_cut_fine * box.h
    k2 = _k2_grid(box.n_coarse, box.H, True)
    xi = np.sqrt(k2) * a_len / 2.0
    S = s2_window(xi)
    with np.errstate(divide="ignore", invalid="ignore"):
        G = -S * S / k2
    G[0, 0, 0] = 0.0
    return G


def short_range_green_continuum(n: int, cell: float, a_len: float, half_last=False, pp_len: float = 0.0):
    """G_s(k) = -(1 - S^2)/k^2 sampled on an n^3 mesh of the given cell size;
    with an extended PP range pp_len > 0 the part inside it is left to the
    pair force: -(S_pp^2 - S^2)/k^2, limit -(a_len^2 - pp_len^2)/30 (P2)."""
    k2 = _k2_grid(n, cell, half_last)
    S = s2_window(np.sqrt(k2) * a_len / 2.0)
    inner = s2_window(np.sqrt(k2) * pp_len / 2.0) ** 2 if pp_len > 0.0 else 1.0
    with np.errstate(divide="ignore", invalid="ignore"):
        G = -(inner - S * S) / k2
    G[0, 0, 0] = -(a_len ** 2 - pp_len ** 2) / 30.0
    return G


def fine_kernel(box: Box, F: int = None) -> np.ndarray:
    """Truncated real-space short-range kernel K_f on the F^3 tile box."""
    F = box.F if F is None else F
    a = box.r_cut_fine
    Gs = short_range_green_continuum(F, box.h, a * box.h, half_last=False, pp_len=box.pp_range * box.h)
    K = np.fft.ifftn(Gs).real
    d = np.fft.fftfreq(F, d=1.0 / F)           # minimum-image offsets in cells
    d2 = d[:, None, None] ** 2 + d[None, :, None] ** 2 + d[None, None, :] ** 2
    K[d2 > a * a] = 0.0
    return K


def fine_green(box: Box, F: int = None) -> np.ndarray:
    """G_f = DFT_F[K_f] in rfftn layout (real, even)."""
    return np.fft.rfftn(fine_kernel(box, F)).real
