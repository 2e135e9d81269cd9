"""Adaptive time step (c chosen every coarse step) on the HIP path vs the FP64
oracle, through the C ABI: populations, elapsed time and link speed bit for
bit in FP64 (the link speed is an order-free max, the rest follows the
shared operation order); FP32 storage within its usual tolerance."""
import numpy as np
import pytest

from paper_2609_35529_amd import workloads as wl
from tests.parity import fp32_error, gpu_solver, run_pair

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True)
def _announce(request):
    print(f"\n[gpu] {request.node.name}", flush=True)
    yield


def _pair(case, steps, kappa=1.5, precision=0, **kw):
    o, g = run_pair(case, 0, precision, **kw)
    o.set_time_stepping(True, kappa)
    g.set_time_stepping(True, kappa)
    if steps:
        o.advance(steps)
        g.advance(steps)
    return o, g


def _bitwise(o, g, case):
    for l in range(case.nlev):
        Fo, Fg = o.get_pop(l), g.get_populations(l)
        assert np.array_equal(Fo, Fg, equal_nan=True), f"level {l}"


def _same_clock(o, g):
    t, c = g.time()
    assert t == o.time() and c == o.link_speed(), (t, o.time(), c, o.link_speed())


def _random_case(nx, ny, nlev, boxes, bc=(0, 0, 0, 0), seed=1, beta=0.8, c=4.0, w=None):
    U = wl.random_state_U(nx, ny, seed=seed)
    states = [U]
    for l in range(1, nlev):
        states.append(wl.prolong_piecewise(states[-1], 2) * (1 + 0.01 * l))
    return wl.Case("rand", nx, ny, 1.0 / max(nx, ny), 2, nlev, 1.4, c, beta, bc, boxes, states, 0,
                   w_inflow=w)


@pytest.mark.parametrize("seed", [0, 2])
def test_quadrant_three_levels(seed):
    case = wl.request_case(dict(n0=48, nlev=3, seed=seed, steps=0))
    o, g = _pair(case, 12)
    _bitwise(o, g, case)
    _same_clock(o, g)


@pytest.mark.parametrize("bc", [(3, 1, 2, 2), (1, 1, 1, 1), (0, 0, 2, 3)])
def test_three_levels_walls_and_inflow(bc):
    """Inflow ghosts take this coarse step's h; every other boundary kind and
    both interfaces follow the changing c."""
    win = np.tile(wl.conserved(1.1, 0.4, -0.1, 1.2).reshape(4), (4, 1))
    case = _random_case(40, 36, 3, [(1, 8, 8, 40, 32), (1, 48, 12, 16, 24), (2, 24, 24, 40, 32)],
                        bc=bc, w=win)
    o, g = _pair(case, 6)
    _bitwise(o, g, case)
    _same_clock(o, g)


def test_fused_substeps_follow_the_time_step():
    """The fused two-sub-step launch of the finest level reads the same h and
    slope ratio as two separate launches."""
    from paper_2609_35529_amd import vlbm
    case = wl.request_case(dict(n0=64, nlev=3, seed=3, steps=0))
    o, g = _pair(case, 0)
    g.set_tuning(256, vlbm.TUNE_FUSE2 | vlbm.TUNE_XCD_ORDER)
    o.advance(10)
    g.advance(10)
    _bitwise(o, g, case)
    _same_clock(o, g)


def test_with_the_adaptive_relaxation():
    case = wl.request_case(dict(n0=48, nlev=3, seed=4, steps=0))
    o, g = _pair(case, 0)
    for s in (o, g):
        s.set_sensor(True, 6.0, 0.4, 0.85)
    o.advance(8)
    g.advance(8)
    _bitwise(o, g, case)
    _same_clock(o, g)


def test_graph_replays_and_toggling(monkeypatch):
    """On a stream the coarse steps replay as graphs (the reduction and the
    scalar update are kernels); switching the adaptive step off returns to the
    parameter c, as in the oracle."""
    import torch
    monkeypatch.setenv("VLBM_GRAPHS", "1")
    stream = torch.cuda.Stream()
    case = wl.request_case(dict(n0=48, nlev=2, seed=5, steps=0))
    o, g = _pair(case, 0, stream=stream)
    o.advance(9)
    g.advance(9)
    _bitwise(o, g, case)
    _same_clock(o, g)
    for s in (o, g):
        s.set_time_stepping(False)
    o.advance(4)
    g.advance(4)
    _bitwise(o, g, case)


@pytest.mark.parametrize("graphs", [False, True])
def test_bound_after_host_changes(monkeypatch, graphs):
    """Each coarse step's last launches carry the CFL bound to the next one.
    A state written by the host (a fast block that raises the bound) and a
    regrid replace it: the next link speed comes from the new state, bit for
    bit as in the oracle, also where the steps replay as graphs."""
    kw = {}
    if graphs:
        import torch
        monkeypatch.setenv("VLBM_GRAPHS", "1")
        kw["stream"] = torch.cuda.Stream()
    case = wl.request_case(dict(n0=48, nlev=2, seed=3, steps=0))
    o, g = _pair(case, 0, **kw)
    o.advance(6)
    g.advance(6)
    _same_clock(o, g)
    c_before = g.time()[1]
    # level 0, 6 x 6 cells in the corner (the patch covers the central half)
    rho, u, p = 1.0, 3.0, 1.0
    U = np.zeros((4, 6, 6))
    U[0], U[1], U[3] = rho, rho * u, p / 0.4 + 0.5 * rho * u * u
    for s in (o, g):
        s.set_state(0, U, 0, 0)
    o.advance(1)
    g.advance(1)
    _same_clock(o, g)
    assert g.time()[1] > c_before
    _bitwise(o, g, case)
    o.advance(5)
    g.advance(5)
    _same_clock(o, g)
    (l, i0, j0, nx, ny), = case.boxes
    for s in (o, g):
        s.regrid([(l, i0 + 4, j0 - 2, nx, ny)])
    for n in (1, 4):
        o.advance(n)
        g.advance(n)
        _same_clock(o, g)
        _bitwise(o, g, case)


@pytest.mark.parametrize("tile,flags", [(256, 20), (1024, 0)])
def test_full_size_quadrant(tile, flags):
    """The 512^2 quadrant with its 512^2 fine patch, kappa = 1.5, in the launch
    configurations the bench times (fused sub-steps in XCD order; unfused
    natural order): 4 coarse steps bit for bit, clock included."""
    case = wl.quadrant(n0=512, seed=0, steps=0)
    o, g = _pair(case, 0)
    g.set_tuning(tile, flags)
    o.advance(4)
    g.advance(4)
    _same_clock(o, g)
    _bitwise(o, g, case)


@pytest.mark.parametrize("precision", [1, 2])
def test_fp32_storage_within_tolerance(precision):
    case = wl.vortex(n0=64, t_end=0.05)
    o, g = _pair(case, case.steps, precision=precision)
    worst = fp32_error(o, g, case)
    assert worst.max() <= 1e-5, worst
    t, c = g.time()
    assert abs(c - o.link_speed()) <= 1e-6 * c and abs(t - o.time()) <= 1e-6 * t


def test_batch_refuses_mixing_fixed_and_adaptive():
    from paper_2609_35529_amd import vlbm
    a = gpu_solver(wl.request_case(dict(n0=32, nlev=1, seed=1, steps=0)))
    b = gpu_solver(wl.request_case(dict(n0=32, nlev=1, seed=2, steps=0)))
    a.set_time_stepping(True, 1.5)
    with pytest.raises(vlbm.VLBMError):
        vlbm.batch_advance([a, b], [1, 1])


def test_batch_equals_alone():
    """Contexts of different sizes, depths and kappas in batched launches:
    each context's populations and clock are bit-identical to advancing it
    alone, and to the oracle; a host-side state change in between is taken
    into the next bound."""
    import torch
    from paper_2609_35529_amd import vlbm
    stream = torch.cuda.Stream()
    specs = ((32, 1, 1, 1.5), (64, 2, 2, 1.2), (48, 3, 3, 2.0))
    steps = [5, 7, 4]
    cases = [wl.request_case(dict(n0=n, nlev=l, seed=sd, steps=0)) for n, l, sd, _ in specs]

    def make(case, kappa):
        g = gpu_solver(case, stream=stream)
        g.set_time_stepping(True, kappa)
        return g

    alone = [make(c, k) for c, (_, _, _, k) in zip(cases, specs)]
    for g, n in zip(alone, steps):
        g.advance(n)
    batched = [make(c, k) for c, (_, _, _, k) in zip(cases, specs)]
    vlbm.batch_advance(batched, steps)
    for case, a, b, (_, _, _, k), n in zip(cases, alone, batched, specs, steps):
        assert a.time() == b.time()
        for l in range(case.nlev):
            assert np.array_equal(a.get_populations(l), b.get_populations(l), equal_nan=True), l
        o = exact_oracle(case, k, n)
        _same_clock(o, b)
        _bitwise(o, b, case)
    # a faster block written into the first context, then one more batched round
    U = np.zeros((4, 4, 4))
    U[0], U[1], U[3] = 1.0, 3.0, 1.0 / 0.4 + 4.5
    alone[0].set_state(0, U, 0, 0)
    batched[0].set_state(0, U, 0, 0)
    for g in alone:
        g.advance(3)
    vlbm.batch_advance(batched, [3, 3, 3])
    for case, a, b in zip(cases, alone, batched):
        assert a.time() == b.time()
        for l in range(case.nlev):
            assert np.array_equal(a.get_populations(l), b.get_populations(l), equal_nan=True), l


def exact_oracle(case, kappa, n):
    from tests import exact
    o = exact.run_oracle(case, steps=0)
    o.set_time_stepping(True, kappa)
    o.advance(n)
    return o
