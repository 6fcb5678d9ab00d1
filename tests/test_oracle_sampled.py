"""Pins of the oracle's sampled evaluators and of the potential energy.

The sampled evaluators (pm.quanta_of_cells, pm.tile_force_sampled,
pm.coarse_force_at) are the reference of every full-size parity test; they
must give, bit for bit, what the whole-box solver gives (which the other pins
of test_oracle_pm.py tie to Ewald sums, momentum conservation and the
analytic split).

The potential energy W = 1/2 sum_i phi_total(x_i) (R19) is pinned by
Parseval's identity, which never interpolates at the particles: with
deposit and gather adjoint (the same CIC weights, R10), sum_i phi(x_i) equals
sum_c M(c) phi(c) for the deposited mass M, and with the mean density
removed (R18) and phi = IDFT(G DFT(rho)) the mesh sum is cell volume times
sum_k G(k) |rho_hat(k)|^2 / n^3 (plus the mean-density term on a tile box,
whose potential does not average to zero).
"""

import numpy as np
import pytest

from cube_inputs import config, lattice_run_state, zeldovich_ics
from oracle import Box, cic, codec, diag, green, pm


def _state(name, **kw):
    spec = config(name).with_(**kw) if kw else config(name)
    box = Box.from_spec(spec).validate()
    pos, vel = zeldovich_ics(spec.n_side, spec.spectral_index, spec.rms_disp, spec.seed, spec.dt)
    return box, codec.compress(box, pos, vel)


def _lattice_state(name):
    """The full-size tests' state layout (lattice plus runs of random cells) on a small box."""
    box = Box.from_spec(config(name)).validate()
    nc = box.n_cells
    counts, m, u = lattice_run_state(nc, [(0, 64), (nc // 3 * 2 // 2 * 2, 128), (nc - 96, 96)], seed=77)
    st = codec.State(box, counts.astype(np.int64), m, u, 2.0 ** -6, int(np.abs(u).max()))
    return box, st


CASES = [("t4", _state), ("c3s", _state), ("t4", _lattice_state)]


@pytest.mark.parametrize("name,make", CASES)
def test_quanta_of_cells_equals_full_decode(name, make):
    box, st = make(name)
    Q = st.quanta()
    off = st.offsets()
    rng = np.random.default_rng(5)
    cells = np.sort(rng.choice(box.n_cells, size=min(box.n_cells, 3000), replace=False))
    idx, Qs = pm.quanta_of_cells(box, st.counts, off, st.m, cells)
    expect_idx = np.concatenate([np.arange(off[c], off[c + 1]) for c in cells])
    assert np.array_equal(idx, expect_idx)
    assert np.array_equal(Qs, Q[expect_idx])
    # every cell at once gives the storage order itself
    idx_all, Q_all = pm.quanta_of_cells(box, st.counts, off, st.m, np.arange(box.n_cells))
    assert np.array_equal(idx_all, np.arange(st.n))
    assert np.array_equal(Q_all, Q)


@pytest.mark.parametrize("name,make", CASES)
def test_sampled_forces_equal_whole_box_solver(name, make):
    box, st = make(name)
    sol = pm.Solver(box)
    _, a_f, a_c = sol.forces(st, parts=True)
    off = st.offsets()
    tiles = range(box.n_tiles) if box.n_tiles <= 8 else [0, 5, 21, box.n_tiles - 1]
    for t in tiles:
        tgt, Qt, af = pm.tile_force_sampled(box, st.counts, off, st.m, t, sol.Gf)
        lo, hi = off[t * box.Tc ** 3], off[(t + 1) * box.Tc ** 3]
        assert np.array_equal(tgt, np.arange(lo, hi))
        assert np.array_equal(Qt, st.quanta()[lo:hi])
        assert np.array_equal(af, a_f[lo:hi])
    Q = st.quanta()
    rho_c = pm.coarse_density(box, Q)
    ac = pm.coarse_force_at(box, rho_c, sol.Gc, Q)
    assert np.array_equal(ac, a_c)


def _green_sum(rho, G, cell):
    """cell^3 sum_c rho(c) phi(c) with phi = irfftn(rfftn(rho) G): Parseval
    over the half spectrum (modes of the last axis other than 0 and n/2
    stand for their conjugates too)."""
    n = rho.shape[0]
    rk = np.fft.rfftn(rho)
    w = np.full(rk.shape[-1], 2.0)
    w[0] = 1.0
    if n % 2 == 0:
        w[-1] = 1.0
    return cell ** 3 * float(np.sum(w * G * np.abs(rk) ** 2)) / n ** 3


@pytest.mark.parametrize("name", ["c1", "t4"])
def test_potential_energy_parseval(name):
    box, st = _state(name)
    sol = pm.Solver(box)
    W = diag.potential_energy(sol, st)
    Q = st.quanta()
    # coarse: the periodic mesh's potential has zero mean, so sum M phi = H^3 sum rho phi
    Wc = 0.5 * _green_sum(pm.coarse_density(box, Q), sol.Gc, box.H)
    # fine: per tile, the targets' mass against the tile's potential
    off = st.offsets()
    Wf = 0.0
    for t in range(box.n_tiles):
        phi, origin = pm.fine_potential_tile(box, Q, st.counts, off, t, sol.Gf)
        tgt = pm.tile_targets(box, off, t)
        M_t = cic.deposit(pm.tile_box_coords(box, Q[tgt], origin), box.F, periodic=box.n_tiles == 1)
        if box.n_tiles == 1:
            rho = M_t / box.h ** 3 - 1.0
            Wf += 0.5 * _green_sum(rho, sol.Gf, box.h)
            # the periodic tile's potential averages to zero, so this is the same sum
            assert abs(float(np.sum(M_t * phi)) - _green_sum(rho, sol.Gf, box.h)) < 1e-9 * abs(Wf)
        else:
            Wf += 0.5 * float(np.sum(M_t * phi))
    expect = Wc + Wf
    assert abs(W - expect) <= 1e-10 * abs(expect)
    # the two meshes' shares are both material, so neither term can be dropped
    assert abs(Wc) > 1e-3 * abs(expect) and abs(Wf) > 1e-3 * abs(expect)


def test_potential_energy_sign_and_scaling():
    """Doubling every density contrast (a clustered copy of the same
    geometry) multiplies the periodic box's W by about four and W is
    negative: gravity binds."""
    spec = config("c1")
    box = Box.from_spec(spec).validate()
    sol = pm.Solver(box)
    Ws = []
    for rms in (0.1, 0.2):
        pos, vel = zeldovich_ics(spec.n_side, spec.spectral_index, rms, spec.seed, spec.dt)
        Ws.append(diag.potential_energy(sol, codec.compress(box, pos, vel)))
    assert Ws[0] < 0 and Ws[1] < 0
    assert 3.0 < Ws[1] / Ws[0] < 5.0
