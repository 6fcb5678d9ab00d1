"""One time step on the compressed state: force, kick, drift, recount, compact.

Integrator (R8): kick-drift leapfrog on (x_n, v_{n-1/2}):
    v_{n+1/2} = v_{n-1/2} + a(x_n) dt,    x_{n+1} = x_n + v_{n+1/2} dt.

Kick and velocity requantisation (R6, R7, R17):
    s' = pow2ceil(h_v M s / 127)            (M = max|u| after the previous kick)
    u' = clamp(rint((u s + a dt) / s'), -127, 127),  M' = max|u'|.

Drift in cell-local quanta (Eq. (2), R15): per axis
    X  = m + 1/2 + ((u' s') (256 / H)) dt
    q  = floor(X),  carry = floor(q / 256),  m' = q - 256 carry,
    n_c' = (n_c + carry) mod N_c.
The product is exact in float64 (an 8-bit integer times powers of two times
the 24-bit dt), so positions never pass through rounded global coordinates.

Recount and compaction (Sec. III-A cell-ordered storage, R16): the new counts
are a histogram of the new cells, and particles are reordered by a stable
counting sort of the old order by new canonical cell.

With the cell-mean velocity codec (Box.vel_codec = 1, vcodec.py V4) the kick
decodes v = v_c + sigma tan(u pi / 255), adds a dt and keeps the result in
FP32; the drift moves by that velocity (X = m + 1/2 + v' (256 / H) dt, exact
in FP64), and after the stable reordering the velocities are re-encoded
against the new cells' means.

In a comoving box (cosmo.py) the same steps run with the kick multiplier
K_n and the FP32 drift multiplier D_n of the step in place of dt.

Pins: the dynamics tests (Zel'dovich plane wave, leapfrog order) exercise the
same kick/drift through the float-state twin in float_mode.py; the compaction
is pinned by brute force (tests/test_oracle_step.py).
"""

import numpy as np

from . import codec, cosmo
from .pm import Solver


def factors(box, state):
    """(kick, drift) multipliers of a step: dt and dt in a static box; the
    comoving K_n and FP32 D_n otherwise (cosmo.py, C3-C4)."""
    if box.comoving:
        return cosmo.step_factors(box, state.step)
    return box.dt, box.dt


def kick(box, state, acc):
    s_new = codec.next_velocity_scale(box, state.s, state.M)
    v = state.u.T.astype(np.float64) * state.s + acc * factors(box, state)[0]
    w = np.rint(v / s_new)
    sat = int(np.count_nonzero(np.abs(w) > 127.0))
    u_new = np.clip(w, -127.0, 127.0).astype(np.int64)       # (N, 3)
    M_new = int(np.max(np.abs(u_new))) if u_new.size else 0
    return u_new, s_new, M_new, sat


def drift(box, state, u_new, s_new):
    """New global quanta (N, 3) and the per-particle carries."""
    m = state.m.T.astype(np.float64)                          # (N, 3)
    D = (u_new.astype(np.float64) * s_new) * (256.0 / box.H) * factors(box, state)[1]
    X = (m + 0.5) + D
    q = np.floor(X).astype(np.int64)
    carry = np.floor_divide(q, 256)
    m_new = q - 256 * carry
    Q_old = state.quanta()
    cell_old = Q_old // 256
    cell_new = np.mod(cell_old + carry, box.n_coarse)
    return 256 * cell_new + m_new, carry


def kick_cell_mean(box, state, acc):
    """V4: decoded velocity plus a dt, held in FP32 (N, 3)."""
    return (state.velocities() + acc * factors(box, state)[0]).astype(np.float32)


def drift_velocity(box, state, v32):
    """Drift by FP32 velocities in cell-local quanta (exact in FP64)."""
    m = state.m.T.astype(np.float64)
    X = (m + 0.5) + v32.astype(np.float64) * (256.0 / box.H) * factors(box, state)[1]
    q = np.floor(X).astype(np.int64)
    carry = np.floor_divide(q, 256)
    cell_new = np.mod(state.quanta() // 256 + carry, box.n_coarse)
    return 256 * cell_new + (q - 256 * carry), carry


def step(solver: Solver, state, workers=None, return_info=False):
    box = solver.box
    acc = solver.forces(state, workers=workers)
    if box.vel_codec == 1:
        v32 = kick_cell_mean(box, state, acc)
        Q_new, carry = drift_velocity(box, state, v32)
        new = codec.build_state_cell_mean(box, Q_new, v32, state.ids, state.step + 1, state.saturations)
        sat = new.saturations - state.saturations
    else:
        u_new, s_new, M_new, sat = kick(box, state, acc)
        Q_new, carry = drift(box, state, u_new, s_new)
        new = codec.build_state(box, Q_new, u_new, s_new, M_new, state.ids,
                                state.step + 1, state.saturations + sat)
    if return_info:
        return new, {"acc": acc, "max_carry": int(np.max(np.abs(carry))) if carry.size else 0,
                     "saturations": sat}
    return new


def run(solver: Solver, state, nsteps: int, workers=None):
    for _ in range(nsteps):
        state = step(solver, state, workers=workers)
    return state
