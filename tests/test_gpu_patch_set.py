"""Batched uneven patches (workloads.patch_set: 100-400 seeded boxes of
16-128 cells on levels 1 and 2 over the shock-bubble problem), every patch of
a level in one launch per phase: bit for bit with the oracle at full size
(three coarse steps, all populations of every level) and on a down-scaled set
with plain, fused and small-level tilings."""
import numpy as np
import pytest

from paper_2609_35529_amd import workloads as wl
from tests import exact
from tests.parity import bitwise_equal, gpu_solver

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True)
def _announce(request):
    print(f"\n[gpu] {request.node.name}", flush=True)
    yield


@pytest.mark.parametrize("tile,flags", [(256, 0), (256, 16), (512, 17 | 2048)])
def test_downscaled_patch_set_matches_oracle(tile, flags):
    case = wl.patch_set(seed=3, nx0=128, ny0=32, np_range=(12, 30), size_range=(8, 32), steps=0)
    assert len([b for b in case.boxes if b[0] == 2]) >= 2
    o = exact.run_oracle(case, steps=0)
    g = gpu_solver(case)
    g.set_tuning(tile, flags)
    for _ in range(3):
        o.advance(2)
        g.advance(2)
        assert bitwise_equal(o, g, case)
    To, Lo = o.totals()
    Tg, Lg = g.totals()
    assert np.all(np.abs((Tg - Lg) - (To - Lo)) <= 1e-13 * np.abs(To).max())


def test_full_size_patch_set_matches_oracle():
    case = wl.patch_set(seed=0, steps=0)
    assert len(case.boxes) >= 100
    o = exact.run_oracle(case, steps=0)
    g = gpu_solver(case)
    g.set_tuning(256, 16)
    o.advance(3)
    g.advance(3)
    assert bitwise_equal(o, g, case)
    assert g.check_health()
