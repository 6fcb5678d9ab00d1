"""Box geometry and the canonical cell order.

Sec. II (two-level decomposition): the volume is cut into cubic tiles; the
short-range PM of a tile runs on a mesh enlarged by the cut-off radius on every
face.  Sec. III-A: particles are stored cell-ordered on the coarse mesh.

Readings: R1 units (lengths in particle spacings), R3 cell-centred
meshes aligned at the origin, R5 canonical order = tile-major (tile index x
fastest), then cells x-fastest inside the tile, R11 tile box F = T + 2b.
"""

from dataclasses import dataclass

import numpy as np


@dataclass(frozen=True)
class Box:
    n_side: int
    tiles_per_dim: int
    fine_per_spacing: int
    coarse_ratio: int
    buffer_fine: int
    r_cut_fine: int
    dt: float
    v_headroom: float = 2.0
    fd_order: int = 2                 # R13: 2- or 4-point gradient on both meshes
    vel_codec: int = 0                # 0: linear bytes (R6); 1: cell means + Eq. (3) bytes (V1-V4)
    comoving: int = 0                 # 1: expanding background, dt is the step in a (C1-C4)
    omega_m: float = 1.0
    omega_l: float = 0.0
    a_start: float = 1.0
    pp_range: int = 0                 # >0: extended PP force within that many fine cells (P1-P4)

    @classmethod
    def from_spec(cls, spec):
        return cls(spec.n_side, spec.tiles_per_dim, spec.fine_per_spacing,
                   spec.coarse_ratio, spec.buffer_fine, spec.r_cut_fine,
                   float(spec.dt), float(spec.v_headroom), int(getattr(spec, "fd_order", 2)),
                   int(getattr(spec, "vel_codec", 0)), int(getattr(spec, "comoving", 0)),
                   # R9: the descriptor carries these as FP32
                   float(np.float32(getattr(spec, "omega_m", 1.0))),
                   float(np.float32(getattr(spec, "omega_l", 0.0))),
                   float(np.float32(getattr(spec, "a_start", 1.0))),
                   int(getattr(spec, "pp_range", 0)))

    # ---- derived sizes -------------------------------------------------
    @property
    def h(self) -> float:             # fine cell size in spacings
        return 1.0 / self.fine_per_spacing

    @property
    def H(self) -> float:             # coarse cell size in spacings
        return self.coarse_ratio / self.fine_per_spacing

    @property
    def n_fine(self) -> int:          # fine cells per box side
        return self.n_side * self.fine_per_spacing

    @property
    def n_coarse(self) -> int:        # N_c
        return self.n_fine // self.coarse_ratio

    @property
    def T(self) -> int:               # tile side, fine cells
        return self.n_fine // self.tiles_per_dim

    @property
    def Tc(self) -> int:              # tile side, coarse cells
        return self.T // self.coarse_ratio

    @property
    def F(self) -> int:               # tile FFT box side, fine cells
        return self.T + 2 * self.buffer_fine

    @property
    def halo_c(self) -> int:          # buffer in coarse cells
        return self.buffer_fine // self.coarse_ratio

    @property
    def n_cells(self) -> int:
        return self.n_coarse ** 3

    @property
    def n_tiles(self) -> int:
        return self.tiles_per_dim ** 3

    def validate(self):
        f, r, b, a = (self.fine_per_spacing, self.coarse_ratio,
                      self.buffer_fine, self.r_cut_fine)
        assert self.n_fine % r == 0 and self.n_fine % self.tiles_per_dim == 0
        assert self.T % r == 0 and b % r == 0
        assert self.fd_order in (2, 4)
        assert self.vel_codec in (0, 1)
        assert self.comoving in (0, 1)
        if self.comoving:
            assert self.omega_m > 0.0 and self.a_start > 0.0
        # P1: partners within one coarse cell, three distinct neighbours per axis
        assert 0 <= self.pp_range <= r and self.pp_range < a
        assert self.pp_range == 0 or self.n_coarse >= 3
        if self.tiles_per_dim == 1:
            assert b == 0 and 2 * a < self.F
        else:
            # R11: a target's CIC nodes lie in [-1, T] of the tile, its
            # gradient reads the potential fd_order/2 cells further out, that
            # potential reads the density a cells further still, and a density
            # cell is complete one cell inside the buffer's edge: a <= b - 3
            # for 2-point gradients, a <= b - 4 for 4-point ones
            assert a <= b - 2 - self.fd_order // 2
            assert self.F // r <= self.n_coarse
        return self

    # ---- canonical order (R5) ------------------------------------------
    def canon(self, cx, cy, cz):
        """Canonical index of coarse cell (cx, cy, cz); arrays allowed."""
        Tc, nt = self.Tc, self.tiles_per_dim
        cx = np.asarray(cx, dtype=np.int64)
        cy = np.asarray(cy, dtype=np.int64)
        cz = np.asarray(cz, dtype=np.int64)
        tile = (cx // Tc) + nt * ((cy // Tc) + nt * (cz // Tc))
        local = (cx % Tc) + Tc * ((cy % Tc) + Tc * (cz % Tc))
        return tile * Tc ** 3 + local

    def cell_of_canon(self, c):
        """Inverse of canon: (cx, cy, cz) arrays."""
        Tc, nt = self.Tc, self.tiles_per_dim
        c = np.asarray(c, dtype=np.int64)
        tile, local = np.divmod(c, Tc ** 3)
        tx = tile % nt
        ty = (tile // nt) % nt
        tz = tile // (nt * nt)
        lx = local % Tc
        ly = (local // Tc) % Tc
        lz = local // (Tc * Tc)
        return tx * Tc + lx, ty * Tc + ly, tz * Tc + lz

    def tile_coords(self, t):
        nt = self.tiles_per_dim
        return t % nt, (t // nt) % nt, t // (nt * nt)
