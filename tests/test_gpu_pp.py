"""GPU parity of the extended PP force (Sec. II optional module; readings
P1-P4 of the oracle's pp.py) through the C ABI.

Forces: relative L2 <= 1e-5 against the oracle (fine mesh with the corrected
kernel, coarse mesh and FP64 pair sums), on Zel'dovich states and on a
clustered state with coincident particles, where close pairs dominate.
Steps: positions within one quantum for >= 99.9% of particles by id.
Full size: sampled tiles of the 1024^3 lattice-with-runs state in the
benchmark's launch configuration."""

import numpy as np
import pytest

from cube_inputs import config, lattice_run_state
from tests.gpu_common import ics, rel_l2

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _zeldovich_state(name, npp):
    import oracle
    from oracle import codec
    spec = config(name).with_(pp_range=npp)
    box = oracle.Box.from_spec(spec).validate()
    pos, vel = ics(name)
    return spec, box, codec.compress(box, pos, vel, with_ids=True)


def _clustered_state(npp, seed=21):
    """c1's geometry with particles in tight clumps; one particle in 64 is
    doubled onto another's exact position."""
    import oracle
    from oracle import codec
    spec = config("c1").with_(pp_range=npp)
    box = oracle.Box.from_spec(spec).validate()
    rng = np.random.default_rng(seed)
    n, L = box.n_side ** 3, float(box.n_side)
    centres = rng.uniform(0, L, (n // 32, 3))
    pos = np.mod(centres[rng.integers(0, centres.shape[0], n)] + 0.4 * rng.standard_normal((n, 3)), L)
    dup = rng.choice(n, n // 64, replace=False)
    pos[dup] = pos[(dup + 1) % n]
    Q = codec.encode_positions(box, pos)
    u = rng.integers(-20, 21, (n, 3)).astype(np.int8)
    st = codec.build_state(box, Q, u, 2.0 ** -6, 20, ids=np.arange(n))
    return spec, box, st


def _gpu_forces(spec, st, batch=3):
    from paper_2003_03931_amd import CubeBox
    with CubeBox(spec, with_ids=True, tiles_per_batch=batch) as g:
        g.set_state(st.counts, st.m, st.u, st.s, st.M, st.ids, st.step)
        return g.forces().cpu().numpy()


@pytest.mark.parametrize("name,npp", [("c1", 4), ("t4", 2)])
def test_pp_forces_match_oracle(name, npp):
    _need_gpu()
    from oracle import pm, pp
    spec, box, st = _zeldovich_state(name, npp)
    a_ref = pm.Solver(box).forces(st, workers=1)
    a_pp = pp.pp_accel(box, st)
    a = _gpu_forces(spec, st)
    err = rel_l2(a, a_ref)
    share = np.linalg.norm(a_pp) / np.linalg.norm(a_ref)
    print(f"{name} pp_range {npp}: force relative L2 {err:.3e}, |PP| / |total| {share:.3e}")
    assert err <= 1e-5
    # the PP part is material in these states
    assert np.linalg.norm(a_pp) > 1e-3 * np.linalg.norm(a_ref)


@pytest.mark.parametrize("npp", [1, 4])
def test_pp_forces_on_clumps_with_coincident_particles(npp):
    """Short (half a spacing, only the own and one neighbour cell per axis)
    and full (one coarse cell) ranges."""
    _need_gpu()
    from oracle import pm, pp
    spec, box, st = _clustered_state(npp)
    a_ref = pm.Solver(box).forces(st, workers=1)
    a_pp = pp.pp_accel(box, st)
    a = _gpu_forces(spec, st)
    err = rel_l2(a, a_ref)
    share = np.linalg.norm(a_pp) / np.linalg.norm(a_ref)
    print(f"clumps, pp_range {npp}: force relative L2 {err:.3e}, |PP| / |total| {share:.3f}")
    assert share > 0.3
    assert err <= 1e-5
    # particles alone in their r_pp neighbourhood get the mesh force only: the
    # doubled ones feel their twin not at all
    assert np.all(np.isfinite(a))


def test_pp_forces_where_neighbourhoods_exceed_the_lds_stage():
    """A quarter of the 32^3 box's particles in one tight clump: the rows
    around it hold more than the 4096 neighbour particles a workgroup stages
    in LDS, so those workgroups read their partners from global memory while
    the others use the staged copy; both against the oracle."""
    _need_gpu()
    import oracle
    from oracle import codec, pm, pp
    spec = config("c1").with_(pp_range=4)
    box = oracle.Box.from_spec(spec).validate()
    rng = np.random.default_rng(22)
    n, L = box.n_side ** 3, float(box.n_side)
    pos = rng.uniform(0, L, (n, 3))
    pos[:n // 4] = np.mod(np.array([9.3, 20.1, 4.7]) + 0.5 * rng.standard_normal((n // 4, 3)), L)
    u = rng.integers(-20, 21, (n, 3)).astype(np.int8)
    st = codec.build_state(box, codec.encode_positions(box, pos), u, 2.0 ** -6, 20, ids=np.arange(n))
    # particles in the 3 x 3 rows of Tc + 2 cells around each row of cells
    Nc, Tc = box.n_coarse, box.Tc
    c = st.counts.reshape(Nc, Nc, Nc)                      # [z][y][x] for one periodic tile
    rows = c.sum(axis=2) + c[:, :, -1] + c[:, :, 0]      # Tc = Nc: the end cells wrap onto the row
    hood = sum(np.roll(np.roll(rows, dz, 0), dy, 1) for dz in (-1, 0, 1) for dy in (-1, 0, 1))
    assert (hood > 4096).sum() > 0 and (hood <= 4096).sum() > 0
    a_ref = pm.Solver(box).forces(st, workers=1)
    a = _gpu_forces(spec, st)
    err = rel_l2(a, a_ref)
    share = np.linalg.norm(pp.pp_accel(box, st)) / np.linalg.norm(a_ref)
    print(f"dense clump: {(hood > 4096).sum()} rows read from global memory, force relative L2 {err:.3e}, "
          f"|PP| / |total| {share:.3f}")
    assert err <= 1e-5


@pytest.mark.parametrize("name,npp,nsteps", [("c1", 4, 2), ("t4", 2, 2)])
def test_pp_steps_match_oracle(name, npp, nsteps):
    _need_gpu()
    from oracle import pm, step
    from paper_2003_03931_amd import CubeBox
    from tests.test_gpu_parity import _compare_by_id
    spec, box, ref = _zeldovich_state(name, npp)
    sol = pm.Solver(box)
    o = ref
    for _ in range(nsteps):
        o = step.step(sol, o, workers=1)
    with CubeBox(spec, with_ids=True, tiles_per_batch=5) as g:
        g.set_state(ref.counts, ref.m, ref.u, ref.s, ref.M, ref.ids, 0)
        g.step(nsteps)
        st = g.get_state()
    assert st["s"] == o.s and st["counts"].sum() == ref.n
    d = _compare_by_id(box, st, o)
    print(f"{name} pp_range {npp}: {nsteps} steps, within 1 quantum {np.mean(d <= 1):.6f}, "
          f"identical {np.mean(d == 0):.6f}")
    assert np.mean(d <= 1) >= 0.999, np.bincount(np.minimum(d, 10))
    assert np.mean(d == 0) >= 0.99


def test_pp_full_size_sampled_cells():
    """1024^3 with pp_range 4 in the benchmark's launch configuration (64
    tiles per batch): the GPU's total force minus its force with the PP
    module off, on the cells of the random runs and their neighbours, against
    the oracle's (fine force with the corrected kernel minus the plain one)
    plus its pair sums.  The coarse force cancels exactly in the difference:
    both boxes share the coarse mesh and its bytes."""
    _need_gpu()
    import oracle
    from oracle import pm, pp, green
    from paper_2003_03931_amd import CubeBox
    spec = config("c3").with_(pp_range=4)
    box = oracle.Box.from_spec(spec).validate()
    box0 = oracle.Box.from_spec(config("c3")).validate()
    Tc = box.Tc
    t = 5 + 16 * (5 + 16 * 5)
    runs = [(t * Tc ** 3 + 12 * Tc * Tc, 4 * Tc * Tc)]
    counts, m, u = lattice_run_state(box.n_cells, runs, seed=3101)
    M = int(np.abs(u.astype(np.int64)).max())
    off = np.zeros(box.n_cells + 1, np.int64)
    np.cumsum(counts, out=off[1:])
    print(f"state: n={counts.sum()} run cells {runs[0][1]}", flush=True)
    rng = np.random.default_rng(3102)
    # run cells (random particles) and a lattice cell next to the run
    cells = np.concatenate([runs[0][0] + rng.choice(runs[0][1], 24, replace=False),
                            [runs[0][0] - 1, runs[0][0] + runs[0][1]]])
    tgt = np.concatenate([np.arange(off[c], off[c + 1]) for c in cells])
    acc = {}
    for key, sp in (("pp", spec), ("plain", config("c3"))):
        g = CubeBox(sp, tiles_per_batch=64)
        g.set_state(counts, m, u, 2.0 ** -6, M)
        a = g.forces()
        acc[key] = a[torch.from_numpy(tgt).to(a.device)].cpu().numpy().astype(np.float64)
        del a
        g.close()
        torch.cuda.empty_cache()
        print(f"gpu forces ({key}) done", flush=True)
    got = acc["pp"] - acc["plain"]
    # oracle: the fine force of tile t with both kernels, then the pair sums
    tg, _, af_pp = pm.tile_force_sampled(box, counts, off, m, t, green.fine_green(box))
    tg0, _, af_0 = pm.tile_force_sampled(box0, counts, off, m, t, green.fine_green(box0))
    assert np.array_equal(tg, tg0)
    pos = {int(p): i for i, p in enumerate(tg)}
    sel = np.array([pos[int(p)] for p in tgt])
    idx, a_pair = pp.pp_accel_cells(box, counts, off, m, cells)
    assert np.array_equal(idx, tgt)
    want = af_pp[sel] - af_0[sel] + a_pair
    full = acc["pp"]
    err = np.linalg.norm(got - want) / np.linalg.norm(full)
    print(f"sampled {tgt.size} particles: |difference error| / |total force| {err:.3e}, "
          f"|PP part| / |total| {np.linalg.norm(want) / np.linalg.norm(full):.3f}", flush=True)
    assert np.linalg.norm(want) > 1e-2 * np.linalg.norm(full)
    assert err <= 1e-5
