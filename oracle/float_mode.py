"""Float-state twin of the PM force and integrator (no fixed-point codec).

Used only to pin the physics: the same two-mesh force (Sec. II, Eq. (1) with
R10-R14) evaluated on float positions, with the whole fine mesh treated as one
periodic mesh, and the kick-drift leapfrog (R8) in float64.  Running the
Zel'dovich plane wave here and again through the compressed step separates
the codec's error from the solver's.

``periodic_fine_green`` embeds the tile box's truncated kernel K_f (a stencil
of radius a) into a periodic mesh of any size; with it the fine force of every
particle equals the tiled force exactly (tiling invariance, R11), which the
tests check.
"""

import numpy as np

from . import cic, green
from .pm import fd_gradient, solve


def periodic_fine_green(box, n: int = None) -> np.ndarray:
    """G on an n^3 periodic fine mesh from the tile-box kernel K_f."""
    n = box.n_fine if n is None else n
    K = green.fine_kernel(box)
    F = K.shape[0]
    a = box.r_cut_fine
    out = np.zeros((n, n, n))
    d = np.arange(-a, a + 1)
    for dx in d:
        for dy in d:
            for dz in d:
                if dx * dx + dy * dy + dz * dz <= a * a:
                    out[dx % n, dy % n, dz % n] = K[dx % F, dy % F, dz % F]
    return np.fft.rfftn(out).real


class FloatSolver:
    def __init__(self, box, Gf_full=None):
        self.box = box
        self.Gc = green.coarse_green(box)
        self.Gf = periodic_fine_green(box) if Gf_full is None else Gf_full

    def parts(self, pos):
        box = self.box
        x = np.asarray(pos, dtype=np.float64)
        rho_c = cic.deposit(x / box.H, box.n_coarse) / box.H ** 3 - 1.0
        g_c = fd_gradient(solve(rho_c, self.Gc), box.H, box.fd_order)
        a_c = cic.gather(g_c, x / box.H).T
        rho_f = cic.deposit(x / box.h, box.n_fine) / box.h ** 3 - 1.0
        g_f = fd_gradient(solve(rho_f, self.Gf), box.h, box.fd_order)
        a_f = cic.gather(g_f, x / box.h).T
        return a_f, a_c

    def forces(self, pos):
        a_f, a_c = self.parts(pos)
        return a_f + a_c


def leapfrog(solver, pos, vel_half, dt: float, nsteps: int, callback=None):
    """KD leapfrog from (x_0, v_{-1/2}); returns the final (x, v)."""
    L = float(solver.box.n_side)
    x = np.array(pos, dtype=np.float64)
    v = np.array(vel_half, dtype=np.float64)
    for i in range(nsteps):
        v = v + solver.forces(x) * dt
        x = np.mod(x + v * dt, L)
        if callback is not None:
            callback(i + 1, x, v)
    return x, v


def leapfrog_comoving(solver, pos, p_half, box, nsteps: int, step0: int = 0):
    """KD leapfrog in the scale factor (cosmo.py C3) from (x at a_step0,
    p at a_step0 - da/2); returns the final (x, p)."""
    from . import cosmo
    L = float(solver.box.n_side)
    x = np.array(pos, dtype=np.float64)
    p = np.array(p_half, dtype=np.float64)
    for i in range(step0, step0 + nsteps):
        K, D = cosmo.step_factors(box, i)
        p = p + solver.forces(x) * K
        x = np.mod(x + p * D, L)
    return x, p
