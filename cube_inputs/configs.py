"""Workload parameters of the synthetic boxes.

Units: lengths in mean inter-particle spacings (box side L = n_side), time in
units of the dynamical time, particle mass 1.

The three single-box workloads:

* ``c1``  -- 32^3 particles, one periodic tile, fine mesh 64^3 (2 cells per
  spacing), coarse mesh 16^3, P(k) ~ k^-2 Zel'dovich ICs at rms displacement
  0.2 spacing, one step.
* ``c2``  -- 256^3 particles, 4^3 tiles of 64^3 particles, fine mesh per tile
  128^3 plus a 16-cell buffer per face (160^3 FFT box), coarse mesh 64^3,
  P(k) ~ k^-2 at rms 0.5, ten steps.
* ``c3``  -- 1024^3 particles, 16^3 tiles of 64^3 particles, same tile box
  as c2, coarse mesh 512^3, P(k) ~ k^-1.5 at rms 2 spacings, twenty steps.

Plus small geometry variants used by the parity tests (several tiles with a
ragged particle distribution at a size the oracle finishes in seconds).
"""

from dataclasses import dataclass, replace

import numpy as np


@dataclass(frozen=True)
class BoxSpec:
    name: str
    n_side: int            # particles per dimension
    tiles_per_dim: int     # n_t
    fine_per_spacing: int  # f: fine cells per particle spacing
    coarse_ratio: int      # r: fine cells per coarse cell
    buffer_fine: int       # b: tile buffer in fine cells (0 when n_t == 1)
    r_cut_fine: int        # a: force-split radius in fine cells
    dt: float              # float32-representable time step
    v_headroom: float      # velocity-scale headroom h_v
    spectral_index: float  # density power-spectrum slope n, P ~ k^n
    rms_disp: float        # rms |psi| of the Zel'dovich displacement
    seed: int
    steps: int
    fd_order: int = 2      # 2- or 4-point central-difference gradients
    vel_codec: int = 0     # 0 linear velocity bytes, 1 cell means + companded bytes
    comoving: int = 0      # 1: expanding background; dt is then the step in the scale factor
    omega_m: float = 1.0   # matter density parameter (comoving runs)
    omega_l: float = 0.0   # cosmological-constant density parameter (comoving runs)
    a_start: float = 1.0   # scale factor of the initial state (comoving runs)
    pp_range: int = 0      # >0: extended PP force within that many fine cells

    def with_(self, **kw):
        return replace(self, **kw)

    @property
    def n_particles(self) -> int:
        return self.n_side ** 3


DT = float(np.float32(0.05))

CONFIGS = {
    "c1": BoxSpec("c1", 32, 1, 2, 4, 0, 12, DT, 2.0, -2.0, 0.2, 1001, 1),
    "c2": BoxSpec("c2", 256, 4, 2, 8, 16, 12, DT, 2.0, -2.0, 0.5, 1002, 10),
    "c3": BoxSpec("c3", 1024, 16, 2, 4, 16, 12, DT, 2.0, -1.5, 2.0, 1003, 20),
    # c2's tile geometry (160^3 tile box, r = 8, b = 16) on a box the oracle
    # runs in seconds: 2^3 tiles of 64^3 particles.
    "c2s": BoxSpec("c2s", 128, 2, 2, 8, 16, 12, DT, 2.0, -2.0, 0.5, 1012, 3),
    # c3's tile geometry (r = 4, b = 16) on 2^3 tiles of 64^3 particles.
    "c3s": BoxSpec("c3s", 128, 2, 2, 4, 16, 12, DT, 2.0, -1.5, 2.0, 1013, 2),
    # the 1024^3 workload's tile geometry (r = 4, b = 16, 160^3 tile box,
    # 8 particles per coarse cell) on 1/64 of its volume: the CPU-baseline sample.
    "c3cpu": BoxSpec("c3cpu", 256, 4, 2, 4, 16, 12, DT, 2.0, -1.5, 2.0, 1033, 1),
    # a small tiled box: 4^3 tiles of 16^3 particles (tile box 32 + 2*16).
    "t4": BoxSpec("t4", 64, 4, 2, 4, 16, 12, DT, 2.0, -2.0, 0.7, 1021, 3),
}


def config(name: str) -> BoxSpec:
    return CONFIGS[name]


def served_box(n_side: int, spectral_index: float, seed: int, name: str = "served", rms_disp: float = 0.5,
               steps: int = 1) -> BoxSpec:
    """A periodic box of the ensemble and serving workloads: f = 2, r = 4
    (coarse mesh at 1/4 of the fine resolution), tiles of 64^3 particles
    (48^3 for a 96^3 box, whose tile box is then 128^3), a 16-cell buffer and
    a 12-cell split radius; one periodic tile at 64^3."""
    if n_side == 64:
        nt, b = 1, 0
    elif n_side == 96:
        nt, b = 2, 16
    else:
        assert n_side % 64 == 0, "sides are 64, 96 or multiples of 64"
        nt, b = n_side // 64, 16
    return BoxSpec(name, n_side, nt, 2, 4, b, 12, DT, 2.0, spectral_index, rms_disp, seed, steps)
