"""GPU: batched ensembles (cube_ensemble_*) against each box run alone.

Boxes of three tile geometries (one periodic 64^3 tile; 96^3 in 48^3 tiles,
tile box 128^3; 128^3 in 64^3 tiles, tile box 160^3) share fine workspaces
by class and their FFT sweeps run as one launch per wave; every box must end
with exactly the bytes of its solo run, under every schedule (streams,
tiles in flight, captured graph or eager launches), after the autotuner,
and when one box halts for the sorted compaction mid-run."""

import numpy as np
import pytest

from cube_inputs import served_box, zeldovich_ics

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

SIDES = [(64, -2.0), (96, -1.5), (128, -2.5), (64, -1.2), (96, -2.2)]


def _specs():
    return [served_box(n, ni, 7100 + i, f"e{i}") for i, (n, ni) in enumerate(SIDES)]


_ICS = {}


def _ics(spec):
    if spec.name not in _ICS:
        _ICS[spec.name] = zeldovich_ics(spec.n_side, spec.spectral_index, spec.rms_disp, spec.seed, spec.dt)
    return _ICS[spec.name]


def _solo(spec, nsteps):
    from paper_2003_03931_amd import CubeBox
    with CubeBox(spec, with_ids=True) as g:
        g.compress(*_ics(spec))
        g.step(nsteps)
        return g.get_state()


_SOLO = {}


def _solo_cached(spec, nsteps):
    key = (spec.name, nsteps)
    if key not in _SOLO:
        _SOLO[key] = _solo(spec, nsteps)
    return _SOLO[key]


def _same(a, b, what):
    for k in ("counts", "m", "u", "ids"):
        assert np.array_equal(a[k], b[k]), f"{what}: {k}"
    assert a["s"] == b["s"] and a["M"] == b["M"] and a["step"] == b["step"], what


def _ensemble(specs, **kw):
    from paper_2003_03931_amd import CubeEnsemble
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    e = CubeEnsemble(specs, with_ids=True, **kw)
    for b, s in zip(e.boxes, specs):
        b.compress(*_ics(s))
    return e


@pytest.mark.parametrize("streams,tiles,graph", [(1, 4, True), (4, 16, True), (2, 8, False), (3, 64, True)])
def test_ensemble_matches_solo_runs(streams, tiles, graph):
    specs = _specs()
    with _ensemble(specs, streams=streams, tiles_in_flight=tiles, use_graph=graph) as e:
        e.step(2)
        e.step(1)
        got = [b.get_state() for b in e.boxes]
        sched = e.schedule()
    assert sched["streams"] == streams and sched["use_graph"] == graph
    for s, g in zip(specs, got):
        _same(g, _solo_cached(s, 3), f"{s.name} ({s.n_side}^3)")


def test_autotuner_keeps_states_and_results():
    specs = _specs()
    with _ensemble(specs) as e:
        before = [b.get_state() for b in e.boxes]
        chosen = e.tune()
        after = [b.get_state() for b in e.boxes]
        for a, b in zip(before, after):
            _same(a, b, "state across tuning")
        assert chosen["streams"] in (1, 2, 4) and chosen["tiles_in_flight"] >= 1
        e.step(3)
        got = [b.get_state() for b in e.boxes]
    for s, g in zip(specs, got):
        _same(g, _solo_cached(s, 3), s.name)


def test_a_halted_box_finishes_alone():
    """Box 1 is forced through the sorted general compaction in its first
    step: it halts inside the graph, is resolved after the replays and
    finishes on its own; every box still ends with its solo bytes."""
    specs = _specs()
    with _ensemble(specs, streams=2, tiles_in_flight=16) as e:
        e.boxes[1].debug_force(2, 1)
        e.step(3)
        got = [b.get_state() for b in e.boxes]
    for s, g in zip(specs, got):
        _same(g, _solo_cached(s, 3), s.name)
