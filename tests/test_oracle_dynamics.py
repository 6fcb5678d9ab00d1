"""Dynamics pins: the Zel'dovich plane wave (R8 leapfrog, static background).

A one-dimensional mode psi = A sin(2 pi q_x / L) e_x grows exactly as e^t in
the continuum before shell crossing.  On the mesh a long mode feels the force
R * psi with a response R < 1 (CIC and differencing); the amplitude then
follows the ODE psi'' = R psi from psi(0) = A, psi'(0) = A:
A(t) = A [cosh(sqrt(R) t) + sinh(sqrt(R) t) / sqrt(R)].
"""

import math

import numpy as np

from cube_inputs import config, plane_wave_ics
from oracle import Box, codec, float_mode, pm, step

L = 32.0
A0 = 0.3


def amplitude(q, x):
    d = np.mod(x[:, 0] - q[:, 0] + L / 2, L) - L / 2
    s = np.sin(2 * np.pi * q[:, 0] / L)
    return np.sum(d * s) / np.sum(s * s)


def setup():
    box = Box.from_spec(config("c1")).validate()
    fs = float_mode.FloatSolver(box)
    q, _, _ = plane_wave_ics(32, A0, box.dt)
    eps = 1e-3
    probe = q.copy()
    probe[:, 0] += eps * np.sin(2 * np.pi * q[:, 0] / L)
    a = fs.forces(probe)
    R = amplitude(q, q + a) / eps
    return box, fs, R, a


def test_mesh_response_of_a_long_mode():
    box, fs, R, a = setup()
    # CIC^2 and the 2-point difference on the 16^3 coarse mesh: ~0.95
    assert 0.93 < R < 0.97
    assert np.max(np.abs(a[:, 1:])) < 1e-14       # no transverse force


def test_plane_wave_growth_float_state():
    box, fs, R, _ = setup()
    q, pos, vel = plane_wave_ics(32, A0, box.dt)
    x, _ = float_mode.leapfrog(fs, pos, vel, box.dt, 10)
    t = 10 * box.dt
    g = amplitude(q, x) / A0
    # (i) continuum growth e^t within 2%
    assert abs(g / math.exp(t) - 1) < 0.02
    # (ii) the mesh-response ODE within 0.2%
    sr = math.sqrt(R)
    assert abs(g / (math.cosh(sr * t) + math.sinh(sr * t) / sr) - 1) < 0.002


def test_leapfrog_is_second_order():
    """Started on the growing mode of the discrete response (small amplitude,
    so the mesh response is linear), the leapfrog error falls 4x per halving
    of dt."""
    box = Box.from_spec(config("c1")).validate()
    fs = float_mode.FloatSolver(box)
    A = 0.01
    q, _, _ = plane_wave_ics(32, A, box.dt)
    probe = q.copy()
    probe[:, 0] += A * np.sin(2 * np.pi * q[:, 0] / L)
    sr = math.sqrt(amplitude(q, q + fs.forces(probe)) / A)
    errs = []
    for n in (5, 10, 20):
        dt = 1.0 / n
        q, pos, _ = plane_wave_ics(32, A, dt)
        vel = np.zeros_like(pos)
        vel[:, 0] = A * sr * math.exp(-sr * dt / 2) * np.sin(2 * np.pi * q[:, 0] / L)
        x, _ = float_mode.leapfrog(fs, pos, vel, dt, n)
        errs.append(amplitude(q, x) / A - math.exp(sr))
    assert 3.6 < errs[0] / errs[1] < 4.4, errs
    assert 3.6 < errs[1] / errs[2] < 4.4, errs


def test_plane_wave_through_compressed_state():
    box, fs, R, _ = setup()
    q, pos, vel = plane_wave_ics(32, A0, box.dt)
    xf, _ = float_mode.leapfrog(fs, pos, vel, box.dt, 10)
    st = codec.compress(box, pos, vel, with_ids=True)
    sol = pm.Solver(box)
    for _ in range(10):
        st = step.step(sol, st)
    gc = amplitude(q[st.ids], st.positions()) / A0
    gf = amplitude(q, xf) / A0
    assert abs(gc / gf - 1) < 0.005          # codec error, not solver error
    assert st.counts.sum() == 32 ** 3
