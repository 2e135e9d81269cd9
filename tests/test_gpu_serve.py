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
