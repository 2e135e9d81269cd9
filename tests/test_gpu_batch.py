"""Batched launches and graph replays give bit-identical results to the plain
per-context path."""
import os

import numpy as np
import pytest

from paper_2609_35529_amd import workloads as wl
from tests.parity import gpu_solver

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True)
def _announce(request):
    print(f"\n[gpu] {request.node.name}", flush=True)
    yield


def _pops(g, nlev):
    return [g.get_populations(l) for l in range(nlev)]


def _same(a, b):
    return all(np.array_equal(x, y, equal_nan=True) for x, y in zip(a, b))


def _mix():
    reqs = [dict(n0=32, nlev=1, seed=1), dict(n0=64, nlev=2, seed=2), dict(n0=48, nlev=3, seed=3),
            dict(n0=16, nlev=2, seed=4), dict(n0=64, nlev=3, seed=5)]
    return [wl.request_case(dict(r, steps=0)) for r in reqs]


@pytest.mark.parametrize("precision", [0, 1, 2])
def test_batch_equals_alone(precision):
    import torch
    stream = torch.cuda.Stream()
    cases = _mix()
    steps = [7, 12, 5, 9, 12]
    alone = []
    for case, n in zip(cases, steps):
        g = gpu_solver(case, precision, stream=stream)
        g.advance(n)
        alone.append(_pops(g, case.nlev))
    from paper_2609_35529_amd import vlbm
    sol = [gpu_solver(case, precision, stream=stream) for case in cases]
    vlbm.batch_advance(sol, steps)
    for g, case, ref, n in zip(sol, cases, alone, steps):
        assert g.steps() == n
        assert _same(_pops(g, case.nlev), ref)


def test_graph_replays_match_eager(monkeypatch):
    """Replays of the captured two-step graph, interleaved with eager work and
    synchronisations, match the eager launches bit for bit after every replay."""
    import torch
    stream = torch.cuda.Stream()
    case = wl.quadrant(n0=64, seed=7, steps=0)
    case = wl.Case(case.name, 64, 64, case.dx0, 2, 3, case.gamma, case.c, case.beta, case.bc,
                   [(1, 32, 32, 64, 64), (2, 80, 80, 64, 64)],
                   [case.states[0], wl.prolong_piecewise(case.states[0], 2),
                    wl.prolong_piecewise(case.states[0], 4)], 0)
    monkeypatch.setenv("VLBM_GRAPHS", "0")
    eager = gpu_solver(case, stream=stream)
    monkeypatch.setenv("VLBM_GRAPHS", "1")
    graph = gpu_solver(case, stream=stream)
    for rep in range(5):
        eager.advance(4)
        graph.advance(4)      # two graph replays
        torch.cuda.synchronize()
        x = torch.ones(1000, device="cuda").sum().item()  # unrelated eager work
        assert x == 1000.0
        assert _same(_pops(eager, 3), _pops(graph, 3)), rep
    eager.advance(3)
    graph.advance(5)          # odd counts: direct step then graph
    eager.advance(2)
    assert _same(_pops(eager, 3), _pops(graph, 3))


def test_set_state_after_steps_keeps_parity():
    case = wl.quadrant(n0=32, seed=2, steps=0)
    a = gpu_solver(case)
    a.advance(3)
    a.set_state(0, case.states[0])
    a.set_state(1, case.states[1])
    b = gpu_solver(case)
    a.advance(5)
    b.advance(5)
    assert _same(_pops(a, 2), _pops(b, 2))


def _mix_fused():
    reqs = [dict(n0=32, nlev=1, seed=11), dict(n0=64, nlev=2, seed=12), dict(n0=48, nlev=3, seed=13),
            dict(n0=16, nlev=2, seed=14), dict(n0=64, nlev=3, seed=15), dict(n0=40, nlev=2, seed=16)]
    return [wl.request_case(dict(r, steps=0)) for r in reqs]


@pytest.mark.parametrize("flags", [16, 16 | 1024, 17 | 1024])
@pytest.mark.parametrize("precision", [0, 2])
def test_fused_and_graph_batches_equal_alone(precision, flags):
    """Contexts of one, two and three levels with fused finest levels (tuning
    flag 16), advanced in batches whose membership changes (all six, then four,
    then two, then all six again), eagerly or as replayed graphs (flag 1024,
    interleaved with unrelated eager work): every context equals the same
    context advanced alone, bit for bit, after every batch."""
    import torch
    from paper_2609_35529_amd import vlbm
    stream = torch.cuda.Stream()
    cases = _mix_fused()
    rounds = [([0, 1, 2, 3, 4, 5], [6, 9, 4, 8, 10, 7]), ([1, 2, 4, 5], [5, 6, 5, 9]),
              ([2, 4], [8, 4]), ([0, 1, 2, 3, 4, 5], [6, 6, 6, 6, 6, 6])]
    alone = []
    for case in cases:
        g = gpu_solver(case, precision, stream=stream)
        g.set_tuning(256, flags & ~1024)
        alone.append(g)
    sol = []
    for case in cases:
        g = gpu_solver(case, precision, stream=stream)
        g.set_tuning(256, flags)
        sol.append(g)
    for ids, steps in rounds:
        for i, n in zip(ids, steps):
            alone[i].advance(n)
        vlbm.batch_advance([sol[i] for i in ids], steps)
        torch.cuda.synchronize()
        assert torch.ones(777, device="cuda").sum().item() == 777.0
        for i in range(len(cases)):
            assert sol[i].steps() == alone[i].steps()
            assert _same(_pops(sol[i], cases[i].nlev), _pops(alone[i], cases[i].nlev)), (ids, i)
