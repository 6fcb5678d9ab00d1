"""Float64 diagnostics of a compressed state.

* mass (exact particle count), momentum sum(v), kinetic energy K = 1/2 sum v^2,
  potential energy W = 1/2 sum phi_total(x_i) (R19);
* matter power spectrum (Sec. IV-C: delta = rho/rho_bar - 1 and
  Delta^2(k) = k^3 P(k) / (2 pi^2)), reading R20: CIC on a diagnostic mesh
  with one cell per spacing, P(k) = L^3 |DFT(delta)|^2 / N_cells^2 averaged in
  shells j = round(|n|) of width k_f = 2 pi / L, for 1 <= j < n/4 (below half
  the diagnostic Nyquist); no deconvolution or shot-noise subtraction.

Pins (tests/test_oracle_diag.py): a single plane-wave density lands in one
shell with the closed-form amplitude; Poisson-random particles give flat
shot noise times the CIC window.
"""

import numpy as np

from . import cic


def moments(state):
    v = state.velocities()
    return {
        "mass": int(state.counts.sum()),
        "momentum": v.sum(axis=0),
        "kinetic": 0.5 * float(np.sum(v * v)),
    }


def potential_energy(solver, state, workers=None):
    _, phi = solver.forces(state, workers=workers, want_phi=True)
    return 0.5 * float(np.sum(phi))


def shell_index(n: int):
    """Integer shell index round(|mode|) of every mode of an n^3 fftn."""
    modes = np.fft.fftfreq(n, d=1.0 / n)
    n2 = modes[:, None, None] ** 2 + modes[None, :, None] ** 2 + modes[None, None, :] ** 2
    return np.floor(np.sqrt(n2) + 0.5).astype(np.int64)


def power_spectrum_from_delta(delta):
    """(k, P, nmodes) of a density-contrast mesh with one cell per spacing."""
    n = delta.shape[0]
    dk = np.fft.fftn(delta)
    p3 = (np.abs(dk) ** 2) / float(n) ** 3  # L^3 / N_cells^2 with L = n
    j = shell_index(n)
    nb = n // 4
    sel = (j >= 1) & (j < nb)
    cnt = np.bincount(j[sel], minlength=nb)[1:nb]
    psum = np.bincount(j[sel], weights=p3[sel], minlength=nb)[1:nb]
    modes = np.fft.fftfreq(n, d=1.0 / n)
    kmag = 2.0 * np.pi / n * np.sqrt(modes[:, None, None] ** 2 + modes[None, :, None] ** 2
                                      + modes[None, None, :] ** 2)
    ksum = np.bincount(j[sel], weights=kmag[sel], minlength=nb)[1:nb]
    with np.errstate(invalid="ignore", divide="ignore"):
        return ksum / cnt, psum / cnt, cnt


def power_spectrum_from_positions(pos, n: int):
    """(k, P, nmodes) for float positions in a periodic box of side n."""
    mass = cic.deposit(np.asarray(pos, dtype=np.float64), n, periodic=True)
    return power_spectrum_from_delta(mass - 1.0)   # rho_bar = 1 per unit cell


def power_spectrum(state):
    return power_spectrum_from_positions(state.positions(), state.box.n_side)
