"""Two-level particle-mesh force (Sec. II).

The force on every particle is the long-range part from one global periodic
coarse mesh plus the short-range part from the fine mesh of the tile the
particle lives in; each tile's fine mesh covers the tile enlarged by a buffer
on every face, and its particles plus the buffer's are the sources (Sec. II,
two-level decomposition; R11).

Per mesh (Eq. (1) applied to the potential, R13):
    rho   = CIC mass / cell volume - 1           (R10, R18: nominal mean removed)
    phi   = IDFT( G * DFT(rho) )                 (R12, R14)
    g     = -(phi(c+e) - phi(c-e)) / (2 * cell)  (2-point central difference)
            or -(8 (phi(c+e) - phi(c-e)) - (phi(c+2e) - phi(c-2e))) / (12 * cell)
                                                 (4-point, the optional R13 variant;
                                                  Box.fd_order picks one for both meshes)
    a     = CIC-gather(g_fine) + CIC-gather(g_coarse)

Positions come straight from the fixed-point state: fine-box coordinates
(Q_box + 1/2) r / 256 and coarse coordinates (Q + 1/2) / 256, both exact.

Removing the nominal mean density 1 instead of the exact box mean changes only
the k = 0 mode, i.e. a constant potential whose difference-gradient is zero.

Pins (tests/test_oracle_pm.py): Eq. (1) equivalence of potential-plus-FD with
the kernel -i sin(k h)/h G (4-point: -i (8 sin(k h) - sin(2 k h))/(6 h) G); exact momentum conservation (pairwise symmetry,
random sets); zero force on a uniform lattice; single-particle force against
the Ewald sum and 1/(4 pi r^2); tiling invariance (tiled fine force equals the
single-periodic-mesh fine force with the same kernel).
"""

import os
from concurrent.futures import ProcessPoolExecutor
import multiprocessing as mp

import numpy as np

from . import cic, green, pp
from .geometry import Box


def fd_gradient(phi, cell: float, order: int = 2) -> np.ndarray:
    """g = -grad phi by 2- or 4-point central differences on a periodic array."""
    if order not in (2, 4):
        raise ValueError("fd order must be 2 or 4")
    g = np.empty((3,) + phi.shape, dtype=np.float64)
    for ax in range(3):
        d1 = np.roll(phi, -1, axis=ax) - np.roll(phi, 1, axis=ax)      # phi(c+e) - phi(c-e)
        if order == 2:
            g[ax] = -d1 / (2.0 * cell)
        else:
            d2 = np.roll(phi, -2, axis=ax) - np.roll(phi, 2, axis=ax)  # phi(c+2e) - phi(c-2e)
            g[ax] = -(8.0 * d1 - d2) / (12.0 * cell)
    return g


def solve(rho, G) -> np.ndarray:
    n = rho.shape[0]
    return np.fft.irfftn(np.fft.rfftn(rho) * G, s=(n, n, n), axes=(0, 1, 2))


# ---------------------------------------------------------------- coarse mesh
def coarse_density(box: Box, Q) -> np.ndarray:
    Xc = (np.asarray(Q, dtype=np.float64) + 0.5) / 256.0
    mass = cic.deposit(Xc, box.n_coarse, periodic=True)
    return mass / box.H ** 3 - 1.0


def coarse_potential(box: Box, Q, Gc=None) -> np.ndarray:
    Gc = green.coarse_green(box) if Gc is None else Gc
    return solve(coarse_density(box, Q), Gc)


# ------------------------------------------------------------------ fine mesh
def _expand_ranges(starts, lens):
    total = int(lens.sum())
    if total == 0:
        return np.zeros(0, dtype=np.int64)
    rep = np.repeat(starts - np.concatenate(([0], np.cumsum(lens)[:-1])), lens)
    return rep + np.arange(total, dtype=np.int64)


def tile_sources(box: Box, state_counts, offsets, t):
    """Indices of the source particles of tile t and their box-relative coarse
    cell offsets (the box origin in coarse cells)."""
    tx, ty, tz = box.tile_coords(t)
    Nc, Tc, hc = box.n_coarse, box.Tc, box.halo_c
    span = box.F // box.coarse_ratio
    origin = np.array([tx * Tc - hc, ty * Tc - hc, tz * Tc - hc]) % Nc
    rng = np.arange(span)
    cz, cy, cx = np.meshgrid((origin[2] + rng) % Nc, (origin[1] + rng) % Nc,
                             (origin[0] + rng) % Nc, indexing="ij")
    cells = box.canon(cx.ravel(), cy.ravel(), cz.ravel())
    idx = _expand_ranges(offsets[cells], state_counts[cells])
    return idx, origin


def tile_box_coords(box: Box, Q_sub, origin) -> np.ndarray:
    """Fine-box coordinates (R11) of particles given their global quanta."""
    Nc = box.n_coarse
    cell = Q_sub // 256
    cb = (cell - origin[None, :]) % Nc
    Qb = cb * 256 + Q_sub % 256
    return (Qb.astype(np.float64) + 0.5) * (box.coarse_ratio / 256.0)


def fine_potential_tile(box: Box, Q, counts, offsets, t, Gf):
    """phi_f on tile t's F^3 box; also returns the box origin (coarse cells)."""
    idx, origin = tile_sources(box, counts, offsets, t)
    X = tile_box_coords(box, Q[idx], origin)
    periodic = box.tiles_per_dim == 1
    mass = cic.deposit(X, box.F, periodic=periodic)
    rho = mass / box.h ** 3 - 1.0
    return solve(rho, Gf), origin


def tile_targets(box: Box, offsets, t):
    lo = offsets[t * box.Tc ** 3]
    hi = offsets[(t + 1) * box.Tc ** 3]
    return np.arange(lo, hi, dtype=np.int64)


def _tile_force(box, Q, counts, offsets, t, Gf, want_phi=False):
    phi, origin = fine_potential_tile(box, Q, counts, offsets, t, Gf)
    tgt = tile_targets(box, offsets, t)
    X = tile_box_coords(box, Q[tgt], origin)
    periodic = box.tiles_per_dim == 1
    acc = cic.gather(fd_gradient(phi, box.h, box.fd_order), X, periodic=periodic).T
    pot = cic.gather(phi, X, periodic=periodic) if want_phi else None
    return tgt, acc, pot


# --------------------------------------------------------- parallel tile loop
_G = {}


def _worker(tiles):
    out = []
    for t in tiles:
        out.append(_tile_force(_G["box"], _G["Q"], _G["counts"], _G["offsets"], t,
                               _G["Gf"], _G["want_phi"]))
    return out


def _fine_all(box, Q, counts, offsets, Gf, want_phi, workers):
    n = Q.shape[0]
    acc = np.zeros((n, 3))
    pot = np.zeros(n) if want_phi else None
    tiles = list(range(box.n_tiles))
    if workers is None:
        workers = int(os.environ.get("CUBE_ORACLE_WORKERS", "1"))
    workers = max(1, min(workers, len(tiles)))
    if workers == 1:
        results = [_tile_force(box, Q, counts, offsets, t, Gf, want_phi) for t in tiles]
    else:
        _G.update(box=box, Q=Q, counts=counts, offsets=offsets, Gf=Gf, want_phi=want_phi)
        chunks = [tiles[i::workers] for i in range(workers)]
        ctx = mp.get_context("fork")
        with ProcessPoolExecutor(max_workers=workers, mp_context=ctx) as ex:
            results = [r for part in ex.map(_worker, chunks) for r in part]
        _G.clear()
    for tgt, a, p in results:
        acc[tgt] = a
        if want_phi:
            pot[tgt] = p
    return acc, pot


# ------------------------------------------- sampled evaluation of large boxes
# The same steps as above, decoding only the particles that a few tiles need,
# for boxes whose full decode would not fit a test's time (R4, R5, R11).
def quanta_of_cells(box: Box, counts, offsets, m, cells):
    """Storage indices and global quanta of the particles of `cells`
    (canonical indices), decoded from counts, offsets and the m planes."""
    cells = np.asarray(cells, dtype=np.int64)
    cnt = np.asarray(counts[cells], dtype=np.int64)
    idx = _expand_ranges(np.asarray(offsets[cells], dtype=np.int64), cnt)
    cx, cy, cz = box.cell_of_canon(np.repeat(cells, cnt))
    Q = np.empty((idx.size, 3), dtype=np.int64)
    Q[:, 0] = 256 * cx + m[0][idx]
    Q[:, 1] = 256 * cy + m[1][idx]
    Q[:, 2] = 256 * cz + m[2][idx]
    return idx, Q


def tile_force_sampled(box: Box, counts, offsets, m, t, Gf):
    """Fine-mesh acceleration of the particles of tile t: (indices, quanta,
    acceleration), with only the tile's sources decoded."""
    tx, ty, tz = box.tile_coords(t)
    Nc, Tc, hc = box.n_coarse, box.Tc, box.halo_c
    span = box.F // box.coarse_ratio
    origin = np.array([tx * Tc - hc, ty * Tc - hc, tz * Tc - hc]) % Nc
    rng = np.arange(span)
    cz, cy, cx = np.meshgrid((origin[2] + rng) % Nc, (origin[1] + rng) % Nc,
                             (origin[0] + rng) % Nc, indexing="ij")
    _, Qs = quanta_of_cells(box, counts, offsets, m, box.canon(cx.ravel(), cy.ravel(), cz.ravel()))
    periodic = box.tiles_per_dim == 1
    rho = cic.deposit(tile_box_coords(box, Qs, origin), box.F, periodic=periodic) / box.h ** 3 - 1.0
    phi = solve(rho, Gf)
    tgt, Qt = quanta_of_cells(box, counts, offsets, m, np.arange(t * Tc ** 3, (t + 1) * Tc ** 3))
    acc = cic.gather(fd_gradient(phi, box.h, box.fd_order), tile_box_coords(box, Qt, origin),
                     periodic=periodic).T
    return tgt, Qt, acc


def coarse_force_at(box: Box, rho_c, Gc, Q):
    """Coarse-mesh acceleration at global quanta Q for a given coarse density
    rho_c (mass per cell volume minus 1)."""
    g = fd_gradient(solve(rho_c, Gc), box.H, box.fd_order)
    return cic.gather(g, (np.asarray(Q, dtype=np.float64) + 0.5) / 256.0, periodic=True).T


# --------------------------------------------------------------------- public
class Solver:
    """Holds the Green's tables of one geometry."""

    def __init__(self, box: Box):
        self.box = box.validate()
        self.Gc = green.coarse_green(box)
        self.Gf = green.fine_green(box)

    def forces(self, state, workers=None, parts=False, want_phi=False):
        """Acceleration (N, 3) in canonical order for a compressed state.

        parts=True returns (a_total, a_fine, a_coarse); want_phi also returns
        the potential at every particle."""
        box = self.box
        Q = state.quanta()
        counts = state.counts
        offsets = state.offsets()
        phi_c = coarse_potential(box, Q, self.Gc)
        Xc = (Q.astype(np.float64) + 0.5) / 256.0
        a_c = cic.gather(fd_gradient(phi_c, box.H, box.fd_order), Xc, periodic=True).T
        a_f, p_f = _fine_all(box, Q, counts, offsets, self.Gf, want_phi, workers)
        a = a_f + a_c
        if box.pp_range:
            a = a + pp.pp_accel(box, state)
        extra = ()
        if want_phi:
            extra = (p_f + cic.gather(phi_c, Xc, periodic=True),)
        if parts:
            return (a, a_f, a_c) + extra
        return (a,) + extra if extra else a
