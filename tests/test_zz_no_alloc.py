"""The allocation-free state read (vlbm_get_state_noalloc) against the
allocating one (vlbm_get_state), through the C ABI: two calls in a row, the
second with a smaller rectangle, on the same and on another context; a
rectangle beyond the static staging is refused before any device work."""
import ctypes as C

import numpy as np
import pytest

from paper_2609_35529_amd import vlbm
from paper_2609_35529_amd import workloads as wl

pytestmark = pytest.mark.gpu


def _read(fn, s, level, i0, j0, nx, ny, ld=None):
    ld = nx if ld is None else ld
    U = np.full((4, ny, ld), 7.0)
    st = fn(s.handle, level, i0, j0, nx, ny, U.ctypes.data_as(C.POINTER(C.c_double)), ld)
    return st, U


def _same(a, b):
    return np.array_equal(a, b, equal_nan=True)


@pytest.mark.parametrize("precision", [vlbm.FP64, vlbm.FP32])
def test_noalloc_read_equals_the_allocating_read(precision):
    print(f"\n[gpu] no-alloc state read, precision {precision}", flush=True)
    case = wl.quadrant(n0=96, seed=2, steps=6)
    s = vlbm.Solver.from_case(case, precision=precision)
    s.advance(case.steps)
    calls = [(0, 0, 0, 96, 96, None),        # whole level 0 (holes read NaN)
             (1, 40, 30, 90, 70, 100),       # part of level 1, a wider host row (ld)
             (1, 0, 0, 20, 12, None)]        # smaller again, outside the patch frame
    for (level, i0, j0, nx, ny, ld) in calls:
        st_a, A = _read(vlbm.vlbm_get_state, s, level, i0, j0, nx, ny, ld)
        st_b, B = _read(vlbm.vlbm_get_state_noalloc, s, level, i0, j0, nx, ny, ld)
        assert st_a == vlbm.VLBM_OK and st_b == vlbm.VLBM_OK, vlbm.vlbm_last_error()
        assert _same(A[:, :, :nx], B[:, :, :nx]), (level, i0, j0, nx, ny)
        assert np.all(B[:, :, nx:] == 7.0)   # beyond nx the caller's row is untouched
    # a second context on the same GPU shares the staging: reads stay correct
    # when calls alternate
    other = vlbm.Solver.from_case(wl.quadrant(n0=64, seed=5, steps=0), precision=precision)
    for _ in range(2):
        for sol, n in ((s, 96), (other, 64)):
            st_a, A = _read(vlbm.vlbm_get_state, sol, 0, 0, 0, n, n)
            st_b, B = _read(vlbm.vlbm_get_state_noalloc, sol, 0, 0, 0, n, n)
            assert st_a == st_b == vlbm.VLBM_OK
            assert _same(A, B)
    s.close()
    other.close()


def test_noalloc_read_refuses_rectangles_beyond_the_staging():
    print("\n[gpu] no-alloc state read: oversize rectangle", flush=True)
    n = 1100  # 1100 x 1000 = 1.1 Mi cells > the staging's 1 Mi cells
    U = wl.random_smooth_U(n, 1000, seed=1)
    s = vlbm.Solver(n, 1000, 1.0 / n, c=4.0, beta=0.8, max_levels=1)
    s.set_hierarchy([])
    s.set_state(0, U)
    st, _ = _read(vlbm.vlbm_get_state_noalloc, s, 0, 0, 0, n, 1000)
    assert st == vlbm.VLBM_EINVAL
    assert b"static staging" in vlbm.vlbm_last_error()
    st, B = _read(vlbm.vlbm_get_state_noalloc, s, 0, 0, 0, 1024, 1000)
    assert st == vlbm.VLBM_OK
    st, A = _read(vlbm.vlbm_get_state, s, 0, 0, 0, 1024, 1000)
    assert st == vlbm.VLBM_OK and _same(A, B)
    s.close()
