"""Fixed-point particle codec (Sec. III-A).

Positions, Eq. (2): each coarse cell is cut into 256 bins per axis; a particle
in cell n_c stores the bin m in one byte and sits at the bin centre.  With the
0-based reading R4 and global quanta Q = 256 n_c + m:

    x = (Q + 1/2) * H / 256,         Q = floor(x * 256 / H) mod (256 N_c).

Storage (Sec. III-A): the m bytes in cell order plus a per-cell particle count
(R5 canonical order, stable inside a cell).

Velocities, default (Box.vel_codec = 0): one signed byte per axis with a
per-box scale (R6, R7) instead of Eq. (3)'s cell-mean-plus-nonlinear form:

    v = u * s,  u = clamp(rint(v / s), -127, 127),  s a power of two,
    s0 = pow2ceil(h_v * max|v| / 127),   s' = pow2ceil(h_v * M * s / 127)

with M = max|u| after the previous kick.  rint is round-half-to-even (R17).
With Box.vel_codec = 1 the state holds Eq. (3)'s form instead (vcodec.py):
per-cell mean velocities v_c plus companded one-byte deviations, and s is the
deviation scale sigma.

Pins (tests/test_oracle_codec.py): exhaustive encode(decode(Q)) == Q for every
quantum, the half-quantum bound on random positions, the velocity half-scale
bound and saturation count, pow2ceil against a brute-force search, brute-force
stable ordering and bincount counts.
"""

from dataclasses import dataclass, field
from typing import Optional

import numpy as np

from .geometry import Box


def pow2ceil(x: float) -> float:
    """Smallest power of two >= x (x > 0), exact via frexp."""
    x = float(x)
    if not x > 0.0:
        raise ValueError("pow2ceil needs a positive argument")
    mant, ex = np.frexp(x)            # x = mant * 2**ex, mant in [0.5, 1)
    if mant == 0.5:
        return float(np.ldexp(1.0, int(ex) - 1))
    return float(np.ldexp(1.0, int(ex)))


def encode_positions(box: Box, pos) -> np.ndarray:
    """Global quanta Q (int64, shape (N, 3)) of float positions (R4)."""
    x = np.asarray(pos, dtype=np.float64)
    q = np.floor(x * (256.0 / box.H)).astype(np.int64)
    return np.mod(q, 256 * box.n_coarse)


def decode_positions(box: Box, Q) -> np.ndarray:
    """Bin-centre positions in spacings, Eq. (2) with 0-based n_c."""
    return (np.asarray(Q, dtype=np.float64) + 0.5) * (box.H / 256.0)


def initial_velocity_scale(box: Box, vel) -> float:
    vmax = float(np.max(np.abs(np.asarray(vel, dtype=np.float64)))) if np.size(vel) else 0.0
    if vmax == 0.0:
        return 1.0
    return pow2ceil(box.v_headroom * vmax / 127.0)


def next_velocity_scale(box: Box, s: float, M: int) -> float:
    """R7: scale for the next kick from the previous max |u| (exact integer)."""
    if M == 0:
        return s
    return pow2ceil(box.v_headroom * float(M) * s / 127.0)


def encode_velocities(v, s: float):
    """u = clamp(rint(v / s)) and the number of saturated components (R6, R17)."""
    w = np.rint(np.asarray(v, dtype=np.float64) / s)
    sat = int(np.count_nonzero(np.abs(w) > 127.0))
    u = np.clip(w, -127.0, 127.0).astype(np.int8)
    return u, sat


@dataclass
class State:
    """Compressed box state: 6 bytes per particle plus per-cell counts."""
    box: Box
    counts: np.ndarray            # int64 [N_c^3], canonical cell order
    m: np.ndarray                 # uint8 [3, N]
    u: np.ndarray                 # int8  [3, N]
    s: float                      # velocity scale (power of two)
    M: int                        # max |u| of the stored velocities
    ids: Optional[np.ndarray] = None   # uint32 [N], test-only identity (R22)
    step: int = 0
    saturations: int = 0
    vc: Optional[np.ndarray] = None    # float32 [N_c^3, 3] cell means (vel_codec 1)

    @property
    def n(self) -> int:
        return self.m.shape[1]

    def offsets(self) -> np.ndarray:
        """Exclusive prefix sum of counts, length N_c^3 + 1 (R5)."""
        off = np.zeros(self.counts.size + 1, dtype=np.int64)
        np.cumsum(self.counts, out=off[1:])
        return off

    def cell_canon(self) -> np.ndarray:
        """Canonical cell index of every stored particle."""
        return np.repeat(np.arange(self.counts.size, dtype=np.int64), self.counts)

    def quanta(self) -> np.ndarray:
        """Global quanta Q (int64 [N, 3]) recovered from order + counts + m."""
        cx, cy, cz = self.box.cell_of_canon(self.cell_canon())
        Q = np.empty((self.n, 3), dtype=np.int64)
        Q[:, 0] = 256 * cx + self.m[0]
        Q[:, 1] = 256 * cy + self.m[1]
        Q[:, 2] = 256 * cz + self.m[2]
        return Q

    def positions(self) -> np.ndarray:
        return decode_positions(self.box, self.quanta())

    def velocities(self) -> np.ndarray:
        if self.vc is not None:
            from . import vcodec
            return vcodec.decode(self.counts, self.vc, self.u.T, self.s)
        return self.u.T.astype(np.float64) * self.s

    def copy(self):
        return State(self.box, self.counts.copy(), self.m.copy(), self.u.copy(),
                     self.s, self.M, None if self.ids is None else self.ids.copy(),
                     self.step, self.saturations, None if self.vc is None else self.vc.copy())


def build_state(box: Box, Q, u, s: float, M: int, ids=None, step=0, saturations=0):
    """Order particles by canonical cell, stably (R5, R16), and count them."""
    Q = np.asarray(Q, dtype=np.int64)
    cells = Q // 256
    key = box.canon(cells[:, 0], cells[:, 1], cells[:, 2])
    order = np.argsort(key, kind="stable")
    counts = np.bincount(key, minlength=box.n_cells).astype(np.int64)
    m = (Q[order] % 256).T.astype(np.uint8)
    uu = np.asarray(u)[order].T.astype(np.int8)       # u given as (N, 3)
    return State(box, counts, np.ascontiguousarray(m), np.ascontiguousarray(uu), s, M,
                 None if ids is None else np.asarray(ids)[order].astype(np.uint32),
                 step, saturations)


def build_state_cell_mean(box: Box, Q, v, ids=None, step=0, saturations=0):
    """Order particles by canonical cell, stably, count them, and encode the
    velocities v (N, 3) against the cells' means (vel_codec 1, V1-V3)."""
    from . import vcodec
    Q = np.asarray(Q, dtype=np.int64)
    cells = Q // 256
    key = box.canon(cells[:, 0], cells[:, 1], cells[:, 2])
    order = np.argsort(key, kind="stable")
    counts = np.bincount(key, minlength=box.n_cells).astype(np.int64)
    m = (Q[order] % 256).T.astype(np.uint8)
    vc, u, sigma, sat = vcodec.encode(counts, np.asarray(v, dtype=np.float64)[order])
    M = int(np.max(np.abs(u.astype(np.int64)))) if u.size else 0
    return State(box, counts, np.ascontiguousarray(m), np.ascontiguousarray(u.T), sigma, M,
                 None if ids is None else np.asarray(ids)[order].astype(np.uint32),
                 step, saturations + sat, vc)


def compress(box: Box, pos, vel, with_ids: bool = False) -> State:
    """Float positions/velocities (any order) -> compressed state."""
    if box.vel_codec == 1:
        ids = np.arange(np.asarray(pos).shape[0], dtype=np.uint32) if with_ids else None
        v32 = np.asarray(vel, dtype=np.float32)     # the library takes FP32 velocities
        return build_state_cell_mean(box, encode_positions(box, pos), v32, ids)
    Q = encode_positions(box, pos)
    s = initial_velocity_scale(box, vel)
    u, sat = encode_velocities(vel, s)          # (N, 3)
    M = int(np.max(np.abs(u.astype(np.int64)))) if u.size else 0
    ids = np.arange(Q.shape[0], dtype=np.uint32) if with_ids else None
    return build_state(box, Q, u, s, M, ids, 0, sat)


def decompress(state: State):
    """Canonical-order float64 positions and velocities."""
    return state.positions(), state.velocities()
