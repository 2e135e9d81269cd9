"""Fused two-sub-step launches of the finest level (tuning flag 16) against
the oracle and against the unfused launches.

The fused launch keeps the arithmetic and the rounding points of two separate
sub-step launches, so FP64 results match the oracle to the FP64 bar and every
precision matches the unfused path bit for bit.
"""
import numpy as np
import pytest

from paper_2609_35529_amd import vlbm
from paper_2609_35529_amd import workloads as wl
from tests import exact
from tests.parity import bitwise_equal, compare_populations, gpu_solver

pytestmark = pytest.mark.gpu
FP64_TOL = 1e-12
FUSE = vlbm.TUNE_FUSE2


@pytest.fixture(autouse=True)
def _announce(request):
    print(f"\n[gpu] {request.node.name}", flush=True)
    yield


def _fused(case, precision=0, flags=FUSE, tile_cells=256):
    g = gpu_solver(case, precision)
    g.set_tuning(tile_cells, flags)
    return g


def _pair(case, steps, flags=FUSE):
    o = exact.run_oracle(case, steps=0)
    g = _fused(case, flags=flags)
    o.advance(steps)
    g.advance(steps)
    return o, g


def _random_case(nx, ny, nlev, boxes, bc=(0, 0, 0, 0), seed=1, beta=0.8, w=None):
    U = wl.random_state_U(nx, ny, seed=seed)
    states = [U]
    for l in range(1, nlev):
        states.append(wl.prolong_piecewise(states[-1], 2) * (1 + 0.01 * l))
    return wl.Case("rand", nx, ny, 1.0 / max(nx, ny), 2, nlev, 1.4, 4.0, beta, bc, boxes, states, 0,
                   w_inflow=w)


def _ledger_matches(o, g):
    To, Lo = o.totals()
    Tg, Lg = g.totals()
    scale = np.abs(To).max()
    assert np.all(np.abs(Tg - To) <= 1e-14 * scale)
    assert np.all(np.abs(Lg - Lo) <= 1e-12 * max(scale, np.abs(Lo).max()))


@pytest.mark.parametrize("seed", [0, 1])
def test_quadrant_fused(seed):
    case = wl.quadrant(n0=48, seed=seed, steps=20)
    o, g = _pair(case, case.steps)
    compare_populations(o, g, case, FP64_TOL)
    assert bitwise_equal(o, g, case)


@pytest.mark.parametrize("bc", [(1, 1, 1, 1), (2, 2, 2, 2), (3, 1, 2, 2), (0, 0, 2, 3)])
def test_fine_level_on_every_side(bc):
    """The finest level touches all four domain sides (boundary tasks of both
    sub-steps, ledger booked by the owning tile only), ragged tile sizes."""
    win = np.tile(wl.conserved(1.1, 0.4, -0.1, 1.2).reshape(4), (4, 1))
    boxes = [(1, 0, 0, 46, 20), (1, 0, 20, 20, 22), (1, 58, 10, 22, 62)]
    case = _random_case(40, 36, 2, boxes, bc=bc, w=win)
    o, g = _pair(case, 7)
    compare_populations(o, g, case, FP64_TOL)
    _ledger_matches(o, g)


def test_three_levels_fused_finest():
    win = np.tile(wl.conserved(1.1, 0.4, -0.1, 1.2).reshape(4), (4, 1))
    case = _random_case(40, 36, 3, [(1, 8, 8, 40, 32), (1, 48, 12, 16, 24),
                                    (2, 24, 24, 40, 32), (2, 96, 28, 30, 22)],
                        bc=(3, 1, 2, 2), w=win)
    o, g = _pair(case, 6)
    compare_populations(o, g, case, FP64_TOL)
    _ledger_matches(o, g)


def test_periodic_wrap_and_staircase():
    """Fine boxes that wrap across the periodic x boundary (ring positions whose
    source is the periodic partner) and touch each other in a staircase."""
    boxes = [(1, 0, 8, 12, 16), (1, 52, 8, 12, 8), (1, 12, 16, 12, 16), (2, 28, 36, 16, 24)]
    case = _random_case(32, 24, 3, boxes, bc=(0, 0, 1, 1))
    o, g = _pair(case, 6)
    compare_populations(o, g, case, FP64_TOL)


def test_fine_strip_across_periodic_domain():
    """A fine band over the full periodic width (wrap partners on the ring) and
    a one-coarse-cell-high periodic strip whose fine level covers the whole
    height (ring sources inside the tile itself)."""
    case = _random_case(24, 20, 2, [(1, 0, 10, 48, 14)], bc=(0, 0, 1, 1))
    o, g = _pair(case, 6)
    compare_populations(o, g, case, FP64_TOL)
    c1 = wl.Case("strip", 40, 1, 1 / 40, 2, 2, 1.4, 4.0, 0.9, (1, 1, 0, 0),
                 [(1, 20, 0, 20, 2)], [wl.random_state_U(40, 1, 5), wl.random_state_U(80, 2, 6)], 0)
    o, g = _pair(c1, 8)
    compare_populations(o, g, c1, FP64_TOL)
    U1 = wl.random_state_U(16, 16, seed=9)
    c2 = wl.Case("cover", 8, 8, 1 / 8, 2, 2, 1.4, 4.0, 0.8, (0,) * 4, [(1, 0, 0, 16, 16)],
                 [U1.reshape(4, 8, 2, 8, 2).mean(axis=(2, 4)), U1], 0)
    o, g = _pair(c2, 5)
    compare_populations(o, g, c2, FP64_TOL)


def test_sod_fused_full_size():
    case = wl.sod_2d()
    o, g = _pair(case, case.steps)
    compare_populations(o, g, case, FP64_TOL)
    _ledger_matches(o, g)


def test_lax_liu_staircase_fused():
    boxes = [(1, 20, 20, 24, 24), (1, 28, 12, 8, 8), (1, 12, 28, 8, 8), (2, 48, 48, 32, 32)]
    case = wl.lax_liu_12(n0=32, boxes=boxes, nlev=3)
    o, g = _pair(case, 25)
    compare_populations(o, g, case, FP64_TOL)


def test_quadrant_full_size_prefix_fused():
    case = wl.quadrant(n0=512, seed=0, steps=4)
    o, g = _pair(case, case.steps, flags=FUSE | vlbm.TUNE_XCD_ORDER | vlbm.TUNE_NT_STORES)
    compare_populations(o, g, case, FP64_TOL)


@pytest.mark.parametrize("precision", [vlbm.FP32, vlbm.FP32_STORAGE])
def test_fused_equals_unfused_bitwise(precision):
    case = wl.quadrant(n0=64, seed=3, steps=15)
    a = gpu_solver(case, precision)
    b = _fused(case, precision)
    a.advance(case.steps)
    b.advance(case.steps)
    for l in range(case.nlev):
        assert np.array_equal(a.get_populations(l), b.get_populations(l), equal_nan=True), l
    assert np.array_equal(a.totals()[0], b.totals()[0])


def test_toggle_mid_run_keeps_history():
    """Switching fusion on and off between steps changes nothing: the tuning
    rebuild keeps the buffers, the flip parity and the previous-step samples."""
    case = _random_case(40, 36, 3, [(1, 8, 8, 40, 32), (2, 24, 24, 40, 32)], bc=(1, 1, 0, 0))
    o = exact.run_oracle(case, steps=0)
    g = gpu_solver(case)
    for k, flags in enumerate([0, FUSE, vlbm.TUNE_NT_STORES, FUSE | vlbm.TUNE_XCD_ORDER,
                               FUSE | vlbm.TUNE_NT_STORES]):
        g.set_tuning(128 if k % 2 else 256, flags)
        o.advance(3)
        g.advance(3)
    compare_populations(o, g, case, FP64_TOL)


def test_regrid_sequence_fused():
    U = wl.random_smooth_U(32, 32, seed=21)
    states = [U, wl.prolong_piecewise(U, 2), wl.prolong_piecewise(wl.prolong_piecewise(U, 2), 2)]
    case = wl.Case("regrid", 32, 32, 1 / 32, 2, 3, 1.4, 4.0, 0.8, (1, 1, 2, 2),
                   [(1, 16, 16, 24, 24), (2, 40, 40, 16, 16)], states, 0)
    o = exact.run_oracle(case, steps=0)
    g = _fused(case)
    o.advance(2)
    g.advance(2)
    for boxes in [[(1, 8, 20, 32, 24)], [(1, 20, 12, 28, 32), (2, 48, 32, 24, 24)], [],
                  [(1, 4, 4, 20, 20), (1, 24, 8, 12, 20), (2, 12, 12, 24, 16)]]:
        o.regrid(boxes)
        g.regrid(boxes)
        o.advance(3)
        g.advance(3)
        sub = wl.Case(case.name, case.nx0, case.ny0, case.dx0, case.r, case.nlev, case.gamma,
                      case.c, case.beta, case.bc, boxes, case.states, 0)
        compare_populations(o, g, sub, FP64_TOL)


def test_batch_rejects_fused_contexts():
    case = wl.quadrant(n0=32, seed=1, steps=2)
    a = gpu_solver(case)
    b = _fused(case)
    with pytest.raises(RuntimeError):
        vlbm.batch_advance([a, b], [1, 1])
    b.set_tuning(256, 0)
    vlbm.batch_advance([a, b], [1, 1])


def test_kernel_times_count_launches():
    """Per-kernel timing records every step launch: r^l launches of level l per
    coarse step, one fused launch per parent step for the finest level."""
    case = wl.quadrant(n0=64, seed=1, steps=6)
    g = gpu_solver(case)
    g.set_profiling(True)
    g.advance(6)
    t = g.kernel_times()
    assert set(t) == {(0, False), (1, False)}
    assert t[(0, False)][1] == 6 and t[(1, False)][1] == 12
    assert t[(0, False)][2] == 6 * g.active_cells(0) and t[(1, False)][2] == 12 * g.active_cells(1)
    assert all(v[0] > 0 for v in t.values())
    g.set_tuning(256, FUSE)
    g.set_profiling(True)
    g.advance(5)
    t = g.kernel_times()
    assert set(t) == {(0, False), (1, True)}
    assert t[(0, False)][1] == 5 and t[(1, True)][1] == 5
    assert t[(1, True)][2] == 5 * g.active_cells(1) and t[(0, False)][2] == 5 * g.active_cells(0)
    g.set_profiling(False)
    g.advance(2)
    assert g.kernel_times() == t
