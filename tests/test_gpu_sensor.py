"""Adaptive relaxation parameter (Sec. 2.2, eq. sensor-B) on the HIP path vs
the FP64 oracle, through the C ABI.

FP64: the state of every level and the beta field of every level's latest step
are bit-identical to the oracle's (both follow one operation order; the only
order-free step, the level-wide max |Q|, is exact). FP32 storage: populations
within 1e-5 relative on smooth cells, beta within 1e-4.
"""
import numpy as np
import pytest

from paper_2609_35529_amd import workloads as wl
from tests.parity import fp32_error, gpu_solver, run_pair

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True)
def _announce(request):
    print(f"\n[gpu] {request.node.name}", flush=True)
    yield


def _pair(case, steps, sensor, precision=0, **kw):
    o, g = run_pair(case, 0, precision, **kw)
    o.set_sensor(True, *sensor)
    g.set_sensor(True, *sensor)
    if steps:
        o.advance(steps)
        g.advance(steps)
    return o, g


def _compare_beta(o, g, case, atol=0.0):
    """beta of every level's latest step at its active cells; returns the
    smallest beta seen (the sensor must have acted somewhere)."""
    lo = np.inf
    for l in range(case.nlev):
        act = ~np.isnan(o.get_pop(l)[0])
        bg = g.get_beta(l)
        assert np.array_equal(~np.isnan(bg), act), f"level {l}: active masks differ"
        if not act.any():
            continue
        bo = o.get_beta(l)
        if atol == 0.0:
            bad = np.nonzero(bg[act] != bo[act])[0]
            assert bad.size == 0, (l, bad.size, bg[act][bad[:4]], bo[act][bad[:4]])
        else:
            assert np.max(np.abs(bg[act] - bo[act])) <= atol, l
        lo = min(lo, float(bg[act].min()))
    return lo


def _bitwise(o, g, case):
    for l in range(case.nlev):
        Fo, Fg = o.get_pop(l), g.get_populations(l)
        assert np.array_equal(Fo, Fg, equal_nan=True), f"level {l}"


def _random_case(nx, ny, nlev, boxes, bc=(0, 0, 0, 0), seed=1, beta=0.8, c=4.0, r=2, w=None):
    U = wl.random_state_U(nx, ny, seed=seed)
    states = [U]
    for l in range(1, nlev):
        states.append(wl.prolong_piecewise(states[-1], r) * (1 + 0.01 * l))
    return wl.Case("rand", nx, ny, 1.0 / max(nx, ny), r, nlev, 1.4, c, beta, bc, boxes, states, 0,
                   w_inflow=w)


def test_sod_two_levels_bit_exact():
    """Sod with an r = 2 patch over the initial jump: outflow in x, periodic in
    y. The sensor lowers beta at the shock; state and beta match bit for bit."""
    case = wl.sod_2d(steps=60)
    o, g = _pair(case, case.steps, (10.0, 0.5, 0.95))
    _bitwise(o, g, case)
    assert _compare_beta(o, g, case) < 0.9


@pytest.mark.parametrize("seed", [0, 3])
def test_quadrant_three_levels_bit_exact(seed):
    """Riemann quadrant with two nested levels: vortical and compressive
    regions, so the gate takes values strictly inside (0, 1)."""
    case = wl.request_case(dict(n0=48, nlev=3, seed=seed, steps=0))
    o, g = _pair(case, 24, (6.0, 0.4, 0.85))
    _bitwise(o, g, case)
    assert _compare_beta(o, g, case) < 0.85


@pytest.mark.parametrize("bc", [(1, 1, 1, 1), (2, 2, 2, 2), (3, 1, 2, 2), (0, 0, 2, 3)])
def test_three_levels_mixed_boundaries_bit_exact(bc):
    """Outflow, reflecting and inflow sides, two patches on level 1 (one at the
    domain edge), one on level 2: neighbours across non-periodic sides, holes
    and the coverage edge stand in as the cell itself."""
    win = np.tile(wl.conserved(1.1, 0.4, -0.1, 1.2).reshape(4), (4, 1))
    case = _random_case(40, 36, 3, [(1, 8, 8, 40, 32), (1, 48, 12, 32, 24),
                                    (2, 24, 24, 40, 32)], bc=bc, w=win)
    o, g = _pair(case, 6, (5.0, 0.3, 0.8))
    _bitwise(o, g, case)
    _compare_beta(o, g, case)
    To, Lo = o.totals()
    Tg, Lg = g.totals()
    scale = np.abs(To).max()
    assert np.all(np.abs(Tg - To) <= 1e-14 * scale)
    assert np.all(np.abs((Tg - Lg) - (To - Lo)) <= 1e-13 * scale)


def test_ragged_single_level_periodic():
    """One periodic level, a size that leaves ragged tiles in both directions."""
    case = wl.Case("u", 67, 45, 1 / 67, 2, 1, 1.4, 4.0, 0.85, (0,) * 4, [],
                   [wl.random_state_U(67, 45, seed=4)], 0)
    o, g = _pair(case, 9, (8.0, 0.5, 0.9))
    _bitwise(o, g, case)
    assert _compare_beta(o, g, case) < 0.9


def test_toggle_mid_run():
    """Constant beta, then the sensor, then constant beta again: the history is
    kept across both switches, as in the oracle."""
    case = _random_case(32, 32, 2, [(1, 16, 16, 32, 32)], seed=5)
    o, g = run_pair(case, 3)
    for s in (o, g):
        s.set_sensor(True, 4.0, 0.5, 0.8)
    o.advance(4)
    g.advance(4)
    _compare_beta(o, g, case)
    for s in (o, g):
        s.set_sensor(False)
    o.advance(2)
    g.advance(2)
    _bitwise(o, g, case)
    assert np.isnan(g.get_beta(0)).all()


def test_regrid_then_sensor_bit_exact():
    """A regrid (merge and split) between sensor steps: new frames get new
    planes, and the first step after it computes beta from the moved state."""
    case = _random_case(32, 32, 3, [(1, 8, 8, 24, 24), (2, 24, 24, 16, 16)], seed=6)
    o, g = _pair(case, 3, (6.0, 0.4, 0.85))
    boxes = [(1, 20, 16, 32, 32), (2, 48, 40, 24, 24)]
    o.regrid(boxes)
    g.regrid(boxes)
    o.advance(4)
    g.advance(4)
    _bitwise(o, g, case)
    _compare_beta(o, g, case)


def test_equal_bounds_reproduce_constant_beta_at_full_size():
    """The 512^2 Riemann quadrant with its r = 2 patch: with beta_min = beta_max = beta
    the sensor path (all three stages, per-cell beta) reproduces the
    constant-beta run bit for bit."""
    case = wl.quadrant(seed=0, steps=0)
    a = gpu_solver(case)
    b = gpu_solver(case)
    b.set_sensor(True, 10.0, case.beta, case.beta)
    a.advance(4)
    b.advance(4)
    for l in range(case.nlev):
        assert np.array_equal(a.get_populations(l), b.get_populations(l), equal_nan=True), l
    bb = b.get_beta(case.nlev - 1)
    assert np.all(bb[~np.isnan(bb)] == case.beta)


def test_full_size_sampled_beta():
    """The 512^2 quadrant with the sensor for 3 coarse steps, FP64: the oracle
    runs the same hierarchy, and beta plus the state agree bit for bit on
    every level (the oracle finishes this in seconds)."""
    case = wl.quadrant(seed=1, steps=0)
    o, g = _pair(case, 3, (8.0, 0.4, case.beta))
    _bitwise(o, g, case)
    assert _compare_beta(o, g, case) < case.beta


def test_batch_equals_alone():
    """Batched launches run the sensor stages per context: bit-identical to
    advancing each context alone; mixing sensor and constant-beta contexts is
    refused."""
    import torch
    from paper_2609_35529_amd import vlbm
    stream = torch.cuda.Stream()
    cases = [wl.request_case(dict(n0=n, nlev=l, seed=s, steps=0))
             for n, l, s in ((32, 1, 1), (64, 2, 2), (48, 3, 3))]
    steps = [5, 7, 4]
    alone = []
    for case, n in zip(cases, steps):
        g = gpu_solver(case, stream=stream)
        g.set_sensor(True, 5.0, 0.4, 0.6)
        g.advance(n)
        alone.append([g.get_populations(l) for l in range(case.nlev)])
    sol = [gpu_solver(case, stream=stream) for case in cases]
    for g in sol:
        g.set_sensor(True, 5.0, 0.4, 0.6)
    vlbm.batch_advance(sol, steps)
    for g, case, ref in zip(sol, cases, alone):
        for l in range(case.nlev):
            assert np.array_equal(g.get_populations(l), ref[l], equal_nan=True)
    sol[1].set_sensor(False)
    with pytest.raises(vlbm.VLBMError):
        vlbm.batch_advance(sol, [1, 1, 1])


@pytest.mark.parametrize("precision", [1, 2])
def test_fp32_storage_within_tolerance(precision):
    """FP32 storage (FP32 or FP64 relaxation arithmetic; the sensor itself is
    FP64): on the smooth isentropic vortex W within 1e-5 of the oracle on smooth
    cells (relative to each component's largest magnitude); on Sod, where the
    sensor acts, beta within 1e-4."""
    case = wl.vortex(n0=64, t_end=0.1)
    o, g = _pair(case, case.steps, (20.0, 0.5, case.beta), precision)
    worst = fp32_error(o, g, case)
    print("fp32 error per level and component:\n", worst)
    assert worst.max() <= 1e-5, worst
    _compare_beta(o, g, case, atol=1e-4)
    case = wl.sod_2d(steps=40)
    o, g = _pair(case, case.steps, (10.0, 0.5, 0.95), precision)
    assert _compare_beta(o, g, case, atol=1e-4) < 0.9


def test_bad_arguments_and_beta_while_off():
    from paper_2609_35529_amd import vlbm
    case = wl.sod_2d(steps=0)
    g = gpu_solver(case)
    assert np.isnan(g.get_beta(0)).all()
    for bad in ((1.0, 0.0, 0.5), (1.0, 0.6, 0.5), (1.0, 0.5, 1.5), (-1.0, 0.5, 0.9)):
        with pytest.raises(vlbm.VLBMError):
            g.set_sensor(True, *bad)
    g.set_sensor(True, 1.0, 0.5, 0.9)
    g.advance(1)
    b = g.get_beta(0)
    assert np.all((b[~np.isnan(b)] >= 0.5) & (b[~np.isnan(b)] <= 0.9))


@pytest.mark.parametrize("tile_cells", [64, 1024])
def test_tile_shapes_and_periodic_seams(tile_cells):
    """64-cell tiles (stacked rectangles) and 1024-cell single-row tiles, with
    boxes across both periodic seams (neighbours found through the wrap), bit
    for bit."""
    case = _random_case(40, 36, 3, [(1, 0, 8, 12, 16), (1, 68, 8, 12, 16), (1, 24, 0, 16, 8),
                                    (1, 24, 64, 16, 8), (2, 4, 20, 12, 20)])
    o, g = _pair(case, 0, (6.0, 0.4, 0.85))
    g.set_tuning(tile_cells, 0)
    o.advance(6)
    g.advance(6)
    _bitwise(o, g, case)
    assert _compare_beta(o, g, case) < 0.85


def test_graph_replays_with_the_sensor(monkeypatch):
    """Pairs of coarse steps replay as graphs (the next-Qmax clear is a kernel
    store in them, no memset)."""
    import torch
    monkeypatch.setenv("VLBM_GRAPHS", "1")
    stream = torch.cuda.Stream()
    case = wl.request_case(dict(n0=48, nlev=3, seed=5, steps=0))
    o, g = _pair(case, 0, (6.0, 0.4, 0.85), stream=stream)
    for n in (8, 5, 6):
        o.advance(n)
        g.advance(n)
        _bitwise(o, g, case)
        _compare_beta(o, g, case)
