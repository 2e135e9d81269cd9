"""FP32 forms of the three-dimensional (D3Q6) path against the FP64 oracle:
float storage with the cell update in FP64, and plain FP32. The hand-off, the
reflux, the ledger and regrid evaluate in FP64 in both forms and round to
float on store. The bar is the 2-D path's: the conserved state within 1e-5 of
each component's scale over the hierarchy (momentum crosses zero, where a
pointwise ratio measures nothing)."""
import numpy as np
import pytest

from paper_2609_35529_amd import workloads as wl
from tests.test_gpu_3d import REGRID_SEQ, _case, _gpu, _oracle

pytestmark = pytest.mark.gpu
TOL = 1e-5


@pytest.fixture(autouse=True)
def _announce(request):
    print(f"\n[gpu] {request.node.name}", flush=True)
    yield


def _forms():
    from paper_2609_35529_amd import vlbm3
    return [vlbm3.FP32_STORAGE, vlbm3.FP32]


def _w_error(o, g, nlev):
    Uo = [o.get_state(l) for l in range(nlev)]
    Ug = [g.get_state(l) for l in range(nlev)]
    scale = [max(float(np.nanmax(np.abs(U[k]))) for U in Uo if not np.isnan(U[k]).all())
             for k in range(5)]
    worst = 0.0
    for l in range(nlev):
        no, ng = np.isnan(Uo[l]), np.isnan(Ug[l])
        assert np.array_equal(no, ng), f"level {l}: active masks differ"
        for k in range(5):
            m = ~no[k]
            if m.any():
                worst = max(worst, float(np.max(np.abs(Ug[l][k][m] - Uo[l][k][m])) / scale[k]))
    return worst


def _pair(case, steps, precision):
    o, g = _oracle(case), _gpu(case, precision=precision)
    o.advance(steps)
    g.advance(steps)
    return o, g


@pytest.mark.parametrize("form", [0, 1])
@pytest.mark.parametrize("bc", [(0,) * 6, (1, 1, 2, 2, 1, 2)])
def test_two_levels_within_fp32_bar(form, bc):
    case = _case(20, 16, 12, 2, [(1, 10, 8, 6, 20, 16, 12)], bc=bc)
    o, g = _pair(case, 8, _forms()[form])
    err = _w_error(o, g, case.nlev)
    assert err <= TOL, err


@pytest.mark.parametrize("form", [0, 1])
def test_three_levels_and_ratio_three(form):
    case = _case(16, 14, 12, 3, [(1, 0, 4, 4, 12, 12, 10), (1, 16, 6, 8, 10, 8, 8),
                                 (2, 8, 12, 12, 12, 10, 8)], bc=(2, 1, 0, 0, 1, 2))
    o, g = _pair(case, 4, _forms()[form])
    assert _w_error(o, g, case.nlev) <= TOL
    case = _case(9, 9, 9, 2, [(1, 6, 6, 6, 12, 12, 9)], r=3)
    o, g = _pair(case, 4, _forms()[form])
    assert _w_error(o, g, case.nlev) <= TOL


@pytest.mark.parametrize("form", [0, 1])
def test_conservation_against_the_ledger(form):
    """Reflecting and outflow walls: what the totals gain equals what the
    ledger booked, up to the float rounding of the stored populations."""
    case = _case(16, 14, 12, 2, [(1, 8, 6, 6, 12, 14, 10)], bc=(1, 2, 2, 1, 2, 2))
    g = _gpu(case, precision=_forms()[form])
    T0, L0 = g.totals()
    g.advance(10)
    T1, L1 = g.totals()
    scale = np.abs(T0).max()
    assert np.all(np.abs((T1 - T0) - (L1 - L0)) <= 1e-5 * scale), ((T1 - T0) - (L1 - L0)) / scale


@pytest.mark.parametrize("form", [0, 1])
def test_regrid_sequence(form):
    case = _case(16, 14, 12, 3, [(1, 4, 4, 4, 12, 12, 10)])
    o, g = _pair(case, 2, _forms()[form])
    for boxes in REGRID_SEQ:
        o.regrid(boxes)
        g.regrid(boxes)
        o.advance(2)
        g.advance(2)
        assert _w_error(o, g, case.nlev) <= TOL, boxes


def test_storage_forms_share_the_float_round_trip():
    """A state set in FP64 reads back through float storage as the float
    rounding of the equilibrium populations; both FP32 forms store the same
    initial populations."""
    from paper_2609_35529_amd import vlbm3
    case = _case(12, 10, 8, 1, [])
    a = _gpu(case, precision=vlbm3.FP32_STORAGE)
    b = _gpu(case, precision=vlbm3.FP32)
    d = _gpu(case)
    Fa, Fb, Fd = a.get_populations(0), b.get_populations(0), d.get_populations(0)
    assert np.array_equal(Fa, Fb)
    assert np.array_equal(Fa, Fd.astype(np.float32).astype(np.float64))


def test_blast_fp32_storage_tracks_fp64():
    """The blast workload at 64^3 with its patch: FP32 storage against the
    GPU's own FP64 run, away from the blast front."""
    from paper_2609_35529_amd import vlbm3
    case = wl.blast3d(n0=64, steps=10)
    a = _gpu(case)
    b = _gpu(case, precision=vlbm3.FP32_STORAGE)
    a.advance(case.steps)
    b.advance(case.steps)
    Ua, Ub = a.get_state(0), b.get_state(0)
    rho = Ua[0]
    m = ~np.isnan(rho)
    # smooth cells: density within 1% of its neighbours along every axis
    for ax in (0, 1, 2):
        for sh in (1, -1):
            nb = np.roll(rho, sh, axis=ax)
            m &= ~np.isnan(nb) & (np.abs(nb - rho) <= 0.01 * np.abs(rho))
    assert m.sum() > 1000
    for k in range(5):
        scale = np.nanmax(np.abs(Ua[k]))
        assert np.max(np.abs(Ub[k][m] - Ua[k][m])) <= TOL * scale, k
