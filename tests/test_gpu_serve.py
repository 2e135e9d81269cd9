"""The continuous-batching server: results identical alone and in the mix,
admission respects the footprint budget, latencies are recorded."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True)
def _announce(request):
    print(f"\n[gpu] {request.node.name}", flush=True)
    yield


def _requests():
    from paper_2609_35529_amd import workloads as wl
    reqs = wl.request_stream(10, rate=200.0, seed=11, sizes=(32, 64, 96), steps_range=(20, 60))
    return reqs


@pytest.mark.parametrize("precision", [0, 1, 2])
def test_served_results_equal_alone(precision):
    import torch
    from paper_2609_35529_amd import serve, vlbm
    stream = torch.cuda.Stream()
    reqs = _requests()
    srv = serve.Server(budget_bytes=2 << 30, precision=precision, quantum=7, stream=stream,
                       keep_states=True)
    mixed, wall = srv.run(reqs, time_scale=0.0)
    alone, _ = serve.run_sequential(reqs, precision=precision, stream=stream, keep_states=True)
    assert len(mixed) == len(alone) == len(reqs)
    by_id = {r.rid: r for r in alone}
    for r in mixed:
        assert np.array_equal(r.state, by_id[r.rid].state, equal_nan=True), r.rid
        assert r.done >= r.admitted >= r.arrival
    stats = serve.summarize(mixed, wall)
    assert stats["solves"] == len(reqs) and stats["p99_latency_s"] >= stats["p50_latency_s"]


def test_admission_respects_budget():
    import torch
    from paper_2609_35529_amd import serve, vlbm, workloads as wl
    stream = torch.cuda.Stream()
    reqs = _requests()
    biggest = max(vlbm.footprint_bytes(wl.request_case(r), vlbm.FP32) for r in reqs)
    srv = serve.Server(budget_bytes=biggest, precision=vlbm.FP32, quantum=9, stream=stream)
    res, _ = srv.run(reqs, time_scale=0.0)   # one resident solve at a time still completes
    assert sorted(r.rid for r in res) == sorted(r["id"] for r in reqs)
    with pytest.raises(RuntimeError):
        serve.Server(budget_bytes=biggest // 4, precision=vlbm.FP32, stream=stream).run(reqs, 0.0)


def test_a_faulty_request_fails_alone():
    """A request whose initial state has a negative density is detected by the
    health scan, reported failed and freed; every other request's state is
    bit-identical to solving it alone."""
    import torch
    from paper_2609_35529_amd import serve
    stream = torch.cuda.Stream()
    reqs = _requests()
    bad = reqs[3]["id"]
    reqs[3] = dict(reqs[3], poison=True)
    srv = serve.Server(budget_bytes=2 << 30, precision=0, quantum=7, stream=stream, keep_states=True,
                       health_every=1)
    mixed, wall = srv.run(reqs, time_scale=0.0)
    assert len(mixed) == len(reqs)
    assert [r.rid for r in mixed if r.failed] == [bad]
    good = [q for q in reqs if q["id"] != bad]
    alone, _ = serve.run_sequential(good, precision=0, stream=stream, keep_states=True)
    by_id = {r.rid: r for r in alone}
    for r in mixed:
        if not r.failed:
            assert np.array_equal(r.state, by_id[r.rid].state, equal_nan=True), r.rid
    stats = serve.summarize(mixed, wall)
    assert stats["failed"] == 1 and stats["solves"] == len(reqs) - 1


@pytest.mark.parametrize("tuning", [None, (256, 16 | 1024)])
def test_served_fp64_mix_matches_oracle_per_request(tuning):
    """Every request of a served FP64 mix (one to three levels, different
    sizes, arrival while others run; plain launches, or fused finest levels
    with replayed graphs) ends in the level-0 state the oracle computes for
    that request alone: NaN holes in the same cells, values within 1e-14
    relative (the populations are bit-identical; the moment sums may round
    in another order)."""
    import torch
    from paper_2609_35529_amd import serve, workloads as wl
    from tests import exact
    stream = torch.cuda.Stream()
    reqs = wl.request_stream(8, rate=400.0, seed=23, sizes=(32, 48, 64), steps_range=(10, 40))
    assert {r["nlev"] for r in reqs} == {1, 2, 3}
    srv = serve.Server(budget_bytes=2 << 30, precision=0, quantum=5, stream=stream,
                       keep_states=True, tuning=tuning)
    mixed, _ = srv.run(reqs, time_scale=0.0)
    by_req = {q["id"]: q for q in reqs}
    assert sorted(r.rid for r in mixed) == sorted(by_req)
    for r in mixed:
        q = by_req[r.rid]
        assert r.steps == q["steps"] and not r.failed
        o = exact.run_oracle(wl.request_case(q), steps=q["steps"])
        Uo = o.get_state(0)
        assert np.array_equal(np.isnan(Uo), np.isnan(r.state)), r.rid
        m = ~np.isnan(Uo)
        err = np.abs(r.state[m] - Uo[m]) / np.maximum(np.abs(Uo[m]), 1e-12)
        assert err.max() <= 1e-14, (r.rid, float(err.max()))
