"""Dynamic AMR on the shock-bubble problem: the GPU tags, clusters and regrids
every few coarse steps; the oracle applies the same boxes and must agree."""
import numpy as np
import pytest

from paper_2609_35529_amd import workloads as wl
from tests import exact
from tests.parity import compare_populations, gpu_solver

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True)
def _announce(request):
    print(f"\n[gpu] {request.node.name}", flush=True)
    yield


@pytest.mark.parametrize("bc_case", ["shock_bubble"])
def test_dynamic_amr_matches_oracle(bc_case):
    case = wl.shock_bubble(nx0=128, ny0=32, nlev=3, steps=0)
    o = exact.run_oracle(wl.Case(case.name, case.nx0, case.ny0, case.dx0, case.r, case.nlev,
                                 case.gamma, case.c, case.beta, case.bc, [], case.states, 0,
                                 w_inflow=case.w_inflow), steps=0)
    g = gpu_solver(case)
    counts = []
    for cycle in range(5):
        g.tag_and_regrid(0.05, buffer=2, min_box=8, max_box=32)
        boxes = g.boxes()
        counts.append(len(boxes))
        o.regrid(boxes)
        sub = wl.Case(case.name, case.nx0, case.ny0, case.dx0, case.r, case.nlev, case.gamma,
                      case.c, case.beta, case.bc, boxes, case.states, 0)
        compare_populations(o, g, sub, 1e-12)
        g.advance(4)
        o.advance(4)
        compare_populations(o, g, sub, 1e-12)
        To, Lo = o.totals()
        Tg, Lg = g.totals()
        assert np.all(np.abs((Tg - Lg) - (To - Lo)) <= 1e-12 * np.abs(To).max())
    assert max(counts) >= 4, counts
    assert g.check_health()
