"""The four-quadrant Riemann problem at full size and full length on the GPU
(512^2 coarse cells, the central r = 2 patch, beta = 0.6, 1000 coarse steps),
quadrant states from seeds 0..7: sampled populations of both levels, the
conserved totals and the boundary ledger against the oracle's values for the
same runs (tests/golden/quadrant512_seed_samples.txt, written by
tests/golden/make_quadrant_beta_sweep.py from the oracle alone), within the
FP64 bar of 1e-12 relative; both levels stay positive."""
import os

import numpy as np
import pytest

from paper_2609_35529_amd import workloads as wl
from tests.parity import gpu_solver

pytestmark = pytest.mark.gpu

SAMPLES = os.path.join(os.path.dirname(__file__), "golden", "quadrant512_seed_samples.txt")
STEPS = 1000
TOL = 1e-12


@pytest.fixture(autouse=True)
def _announce(request):
    print(f"\n[gpu] {request.node.name}", flush=True)
    yield


def _records():
    cells, totals = {}, {}
    for line in open(SAMPLES):
        if line.startswith("#") or not line.strip():
            continue
        f = line.split()
        seed = int(f[0])
        if f[1] == "totals":
            totals[seed] = (np.array([float(x) for x in f[2:6]]), np.array([float(x) for x in f[6:10]]))
        else:
            cells.setdefault(seed, []).append((int(f[1]), int(f[2]), int(f[3]),
                                               np.array([float(x) for x in f[4:20]])))
    return cells, totals


CELLS, TOTALS = _records()


@pytest.mark.parametrize("seed", range(8))
def test_full_size_full_length_seed(seed):
    case = wl.quadrant(n0=512, seed=seed, steps=0, beta=0.6, kappa=1.5)
    g = gpu_solver(case)
    g.advance(STEPS)
    assert g.check_health()
    for level, i, j, fo in CELLS[seed]:
        fg = g.get_populations(level, i, j, 1, 1).reshape(16)
        scale = np.maximum(np.abs(fo), 1e-3 * np.abs(fo).max())
        err = float(np.max(np.abs(fg - fo) / scale))
        assert err <= TOL, (level, i, j, err)
    T, L = g.totals()
    To, Lo = TOTALS[seed]
    assert np.allclose(T, To, rtol=TOL, atol=TOL * np.abs(To).max()), (T, To)
    assert np.allclose(L, Lo, rtol=1e-10, atol=TOL * np.abs(To).max()), (L, Lo)
