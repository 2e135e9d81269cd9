"""Kelvin-Helmholtz shear layer with dynamic refinement (three levels at
ratio 2 tracking the layer by tagging, clustering, merge and split).

Down-scaled full problem: GPU against the oracle, element by element, through
every regrid. Full-size strip (one GPU's share of the 4096^2 problem): the
properties that hold at any size (conservation through the boundary ledger,
health, the levels reached)."""
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


def _dynamic(case):
    return wl.Case(case.name, case.nx0, case.ny0, case.dx0, case.r, case.nlev, case.gamma, case.c,
                   case.beta, case.bc, [], [case.states[0]] + [None] * (case.nlev - 1), 0,
                   w_inflow=case.w_inflow)


def test_kh_three_refinement_levels_match_oracle():
    case = _dynamic(wl.kelvin_helmholtz(n0=64, seed=2, nlev=4, steps=0))
    o = exact.run_oracle(case, steps=0)
    g = gpu_solver(case)
    deepest = 0
    T0, _ = o.totals()
    for cycle in range(6):
        g.tag_and_regrid(0.05, buffer=2, min_box=8, max_box=32)
        boxes = g.boxes()
        deepest = max([deepest] + [b[0] for b in boxes])
        o.regrid(boxes)
        sub = wl.Case(case.name, case.nx0, case.ny0, case.dx0, case.r, case.nlev, case.gamma,
                      case.c, case.beta, case.bc, boxes, case.states, 0)
        compare_populations(o, g, sub, 1e-12)
        g.advance(5)
        o.advance(5)
        compare_populations(o, g, sub, 1e-12)
        To, _ = o.totals()
        Tg, _ = g.totals()
        scale = np.abs(T0).max()
        assert np.all(np.abs(Tg - To) <= 1e-14 * scale)
        assert np.all(np.abs(To - T0) <= 1e-13 * scale)  # periodic: exact conservation
    assert deepest == 3
    assert g.check_health()


def test_kh_strip_full_size_conserves():
    """4096 x 512 strip of the 4096^2 problem around the layer at y = 0.25,
    levels 1-3 built by tagging, 10 coarse steps with a regrid after 5."""
    case = wl.kelvin_helmholtz_strip()
    g = gpu_solver(case, precision=0)
    for _ in range(case.nlev - 1):
        g.tag_and_regrid(0.05, buffer=4, min_box=16, max_box=128)
    assert max(b[0] for b in g.boxes()) == 3
    T0, L0 = g.totals()
    g.advance(5)
    g.tag_and_regrid(0.05, buffer=4, min_box=16, max_box=128)
    g.advance(5)
    T1, L1 = g.totals()
    scale = np.abs(T0).max()
    assert np.all(np.abs((T1 - T0) - (L1 - L0)) <= 1e-12 * scale), (T1 - T0, L1 - L0)
    assert g.check_health()
    assert all(g.active_cells(l) > 0 for l in range(case.nlev))


def _kh_dynamic(n0):
    return wl.kelvin_helmholtz(n0=n0, seed=0, nlev=4, steps=0, dynamic=True)


def test_kh_downscaled_bench_settings_match_oracle():
    """The 4096^2 problem down-scaled to 128^2 coarse (finest level 1024^2),
    with the bench's refinement settings (threshold 0.01, buffer 4, boxes
    16..128, a regrid every 5 coarse steps) and launch tuning (512-cell tiles,
    non-temporal stores, fused sub-steps of the finest level, smaller tiles on
    levels with few of them): bit for bit with the oracle after every regrid
    and the steps that follow."""
    case = _kh_dynamic(128)
    g = gpu_solver(case)
    g.set_tuning(512, 17 | 2048)
    for _ in range(case.nlev - 1):
        g.tag_and_regrid(0.01, buffer=4, min_box=16, max_box=128)
    o = exact.run_oracle(case, steps=0)
    o.regrid(g.boxes())
    assert max(b[0] for b in g.boxes()) == 3
    for cycle in range(4):
        sub = wl.Case(case.name, case.nx0, case.ny0, case.dx0, case.r, case.nlev, case.gamma,
                      case.c, case.beta, case.bc, g.boxes(), case.states, 0)
        compare_populations(o, g, sub, 0.0)
        g.advance(5)
        o.advance(5)
        compare_populations(o, g, sub, 0.0)
        g.tag_and_regrid(0.01, buffer=4, min_box=16, max_box=128)
        o.regrid(g.boxes())


def test_kh4096_full_size_prefix():
    """The full 4096^2 problem in the bench's launch configuration: levels 1-3
    from tagging, 10 coarse steps with a regrid after 5. Periodic, so the
    totals are conserved to round-off; every cell stays healthy; and the
    fused launch configuration equals the unfused one with other tiles, bit
    for bit (the FP64 contract makes every launch configuration identical)."""
    case = _kh_dynamic(4096)
    runs = []
    for tile, flags in ((512, 17 | 2048), (256, 0)):
        g = gpu_solver(case)
        g.set_tuning(tile, flags)
        for _ in range(case.nlev - 1):
            g.tag_and_regrid(0.01, buffer=4, min_box=16, max_box=128)
        T0, _ = g.totals()
        g.advance(5)
        g.tag_and_regrid(0.01, buffer=4, min_box=16, max_box=128)
        g.advance(5)
        T1, _ = g.totals()
        scale = np.abs(T0).max()
        assert np.all(np.abs(T1 - T0) <= 1e-14 * scale), (T1 - T0) / scale
        assert g.check_health()
        assert max(b[0] for b in g.boxes()) == 3
        runs.append(g)
    a, b = runs
    assert a.boxes() == b.boxes()
    assert np.array_equal(a.get_state(0), b.get_state(0), equal_nan=True)
    for l in range(1, case.nlev):  # the refined bands (whole levels would not fit in host memory)
        N = case.nx0 * 2 ** l
        for yc in (N // 4, 3 * N // 4):
            Sa = a.get_state(l, 0, yc - 64, N, 128)
            Sb = b.get_state(l, 0, yc - 64, N, 128)
            assert np.isfinite(Sa).any()
            assert np.array_equal(Sa, Sb, equal_nan=True), (l, yc)
    for g in runs:
        g.close()
