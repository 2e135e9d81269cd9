"""Per-step metrics lines (JSON) of a running solve: totals, ledger, the
conservation defect against the ledger, health and kernel times."""
import io
import json

import numpy as np
import pytest

from paper_2609_35529_amd import workloads as wl
from tests.parity import gpu_solver

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True)
def _announce(request):
    print(f"\n[gpu] {request.node.name}", flush=True)
    yield


def test_logged_run_balances_and_equals_an_unlogged_run():
    from paper_2609_35529_amd import metrics
    U = wl.random_state_U(40, 36, seed=3)
    states = [U, wl.prolong_piecewise(U, 2), wl.prolong_piecewise(wl.prolong_piecewise(U, 2), 2)]
    case = wl.Case("walls", 40, 36, 1 / 40, 2, 3, 1.4, 4.0, 0.8, (1, 2, 1, 2),
                   [(1, 8, 8, 40, 32), (2, 24, 24, 40, 32)], states, 0)
    g, ref = gpu_solver(case), gpu_solver(case)
    buf = io.StringIO()
    recs = metrics.run_logged(g, 10, 4, buf)
    lines = [json.loads(x) for x in buf.getvalue().splitlines()]
    assert lines == recs and [r["coarse_steps"] for r in lines] == [4, 8, 10]
    for r in lines:
        assert r["healthy"]
        assert max(abs(d) for d in r["defect_rel"]) <= 1e-13
        assert set(r["kernel_ms"]) >= {"0", "1"}
    assert any(abs(x) > 0 for x in lines[-1]["ledger"])  # the walls booked something
    ref.advance(10)  # logging changes nothing
    for l in range(case.nlev):
        assert np.array_equal(g.get_populations(l), ref.get_populations(l), equal_nan=True)
