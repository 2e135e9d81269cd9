"""Device memory through the C ABI: the library's blocks come from the
caller (PyTorch's caching allocator via vlbm_bind_allocator, or one bound
tensor via vlbm_bind_pool); results do not depend on where memory comes from,
and a caller that cannot supply memory gets VLBM_ENOMEM."""
import ctypes as C

import numpy as np
import pytest
import torch

from paper_2609_35529_amd import vlbm
from paper_2609_35529_amd import workloads as wl

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True)
def _announce(request):
    print(f"\n[gpu] {request.node.name}", flush=True)
    yield


def _run(memory=None, pool_bytes=None):
    case = wl.quadrant(n0=96, seed=4, steps=0)
    kw = {"memory": memory} if memory else {}
    s = vlbm.Solver.from_case(case, pool_bytes=pool_bytes, **kw)
    s.set_tuning(256, 16)
    s.advance(4)
    s.regrid([(1, 32, 32, 80, 64), (1, 120, 100, 40, 48)])
    s.advance(3)
    s.tag_and_regrid(0.05, buffer=2, min_box=8, max_box=32)
    s.advance(3)
    out = [s.get_populations(l) for l in range(case.nlev)], s.totals(), s.boxes(), s.memory
    return s, out


def test_results_do_not_depend_on_the_allocator():
    torch.cuda.synchronize()
    before = torch.cuda.memory_allocated()
    s_t, (Ft, Tt, Bt, mt) = _run()              # PyTorch's caching allocator (default)
    assert mt == "torch"
    assert torch.cuda.memory_allocated() - before >= s_t._alloc.bytes_in_use > 0
    s_l, (Fl, Tl, Bl, ml) = _run(memory="library")
    assert ml == "library"
    s_p, (Fp, Tp, Bp, mp) = _run(pool_bytes=256 << 20)
    assert mp == "pool"
    assert Bt == Bl == Bp
    for l in range(len(Ft)):
        assert np.array_equal(Ft[l], Fl[l], equal_nan=True)
        assert np.array_equal(Ft[l], Fp[l], equal_nan=True)
    for a, b in zip(Tt, Tl):
        assert np.array_equal(a, b)
    held = s_t._alloc
    s_t.close()
    assert held.bytes_in_use == 0 and not held.live  # every block went back to PyTorch
    s_l.close()
    s_p.close()


def test_exhausted_pool_and_failing_allocator_give_enomem():
    case = wl.quadrant(n0=256, seed=1, steps=0)
    small = vlbm.torch_pool(1 << 20)
    p = vlbm.make_params(case.nx0, case.ny0, case.dx0, case.gamma, case.c, case.beta, case.r,
                         case.nlev, case.bc, None, vlbm.FP64)
    arr, n = vlbm.make_boxes(case.boxes)
    h = C.c_void_p()
    assert vlbm.vlbm_create(C.byref(p), None, C.byref(h)) == vlbm.VLBM_OK
    assert vlbm.vlbm_bind_pool(h, C.c_void_p(small.data_ptr()), small.numel()) == vlbm.VLBM_OK
    assert vlbm.vlbm_set_hierarchy(h, arr, n) == vlbm.VLBM_ENOMEM
    vlbm.vlbm_destroy(h)
    # an allocator that gives out two blocks, then none
    live = {}

    def alloc(nbytes, user):
        if len(live) >= 2:
            return None
        t = torch.empty(int(nbytes), dtype=torch.uint8, device="cuda")
        live[t.data_ptr()] = t
        return t.data_ptr()

    def free(ptr, user):
        live.pop(ptr, None)

    a_cb, f_cb = vlbm.ALLOC_FN(alloc), vlbm.FREE_FN(free)
    h = C.c_void_p()
    assert vlbm.vlbm_create(C.byref(p), None, C.byref(h)) == vlbm.VLBM_OK
    assert vlbm.vlbm_bind_allocator(h, a_cb, f_cb, None) == vlbm.VLBM_OK
    assert vlbm.vlbm_bind_pool(h, C.c_void_p(small.data_ptr()), small.numel()) == vlbm.VLBM_ESTATE
    assert vlbm.vlbm_set_hierarchy(h, arr, n) == vlbm.VLBM_ENOMEM
    vlbm.vlbm_destroy(h)
    assert not live  # destroy handed back what it held
