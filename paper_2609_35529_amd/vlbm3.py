"""Python binding of the three-dimensional (D3Q6) path of ``libvlbm.so`` (the C
ABI of ``include/vlbm3.h``).

Argument marshalling only: every step runs in the library's HIP kernels. The
library is loaded by ``vlbm`` (which raises ``ImportError`` if it is not
built); there is no CPU fallback.
"""
from __future__ import annotations

import ctypes as C
from typing import Iterable, Optional, Sequence

import numpy as np

from . import vlbm as _v

_lib = _v._lib
LIB_PATH = _v.LIB_PATH
check = _v.check
VLBMError = _v.VLBMError
PERIODIC, OUTFLOW, REFLECT = _v.PERIODIC, _v.OUTFLOW, _v.REFLECT
MAX_LEVELS = 6
TUNE_NT_STORES = 1
FP64, FP32, FP32_STORAGE = _v.FP64, _v.FP32, _v.FP32_STORAGE


class vlbm3_params(C.Structure):
    _fields_ = [("nx0", C.c_int), ("ny0", C.c_int), ("nz0", C.c_int), ("dx0", C.c_double),
                ("bc", C.c_int * 6), ("gamma", C.c_double), ("c", C.c_double),
                ("beta", C.c_double), ("r", C.c_int), ("max_levels", C.c_int),
                ("precision", C.c_int)]


class vlbm3_box(C.Structure):
    _fields_ = [("level", C.c_int), ("i0", C.c_int), ("j0", C.c_int), ("k0", C.c_int),
                ("nx", C.c_int), ("ny", C.c_int), ("nz", C.c_int)]


_P = C.c_void_p
_D = C.POINTER(C.c_double)
_st = C.c_int


def _sig(name, res, args):
    f = getattr(_lib, name)
    f.restype = res
    f.argtypes = args
    return f


_rect = [_P, C.c_int, C.c_int, C.c_int, C.c_int, C.c_int, C.c_int, C.c_int, _D]
vlbm3_create = _sig("vlbm3_create", _st, [C.POINTER(vlbm3_params), _P, C.POINTER(_P)])
vlbm3_destroy = _sig("vlbm3_destroy", None, [_P])
vlbm3_footprint_bytes = _sig("vlbm3_footprint_bytes", C.c_size_t,
                             [C.POINTER(vlbm3_params), C.POINTER(vlbm3_box), C.c_int])
vlbm3_set_hierarchy = _sig("vlbm3_set_hierarchy", _st, [_P, C.POINTER(vlbm3_box), C.c_int])
vlbm3_regrid = _sig("vlbm3_regrid", _st, [_P, C.POINTER(vlbm3_box), C.c_int])
vlbm3_set_state = _sig("vlbm3_set_state", _st, _rect)
vlbm3_set_populations = _sig("vlbm3_set_populations", _st, _rect)
vlbm3_get_state = _sig("vlbm3_get_state", _st, _rect)
vlbm3_get_populations = _sig("vlbm3_get_populations", _st, _rect)
vlbm3_advance = _sig("vlbm3_advance", _st, [_P, C.c_int])
vlbm3_conserved_totals = _sig("vlbm3_conserved_totals", _st, [_P, _D, _D])
vlbm3_set_tuning = _sig("vlbm3_set_tuning", _st, [_P, C.c_int, C.c_int])
vlbm3_set_profiling = _sig("vlbm3_set_profiling", _st, [_P, C.c_int])
vlbm3_kernel_times = _sig("vlbm3_kernel_times", _st, [_P, _D, C.POINTER(C.c_long), _D])
vlbm3_active_cells = _sig("vlbm3_active_cells", C.c_long, [_P, C.c_int])
vlbm3_sync = _sig("vlbm3_sync", _st, [_P])
vlbm3_tag = _sig("vlbm3_tag", _st, [_P, C.c_int, C.c_double, C.POINTER(C.c_uint8)])
vlbm3_tag_and_regrid = _sig("vlbm3_tag_and_regrid", _st, [_P, C.c_double, C.c_int, C.c_int, C.c_int])
vlbm3_get_boxes = _sig("vlbm3_get_boxes", _st, [_P, C.POINTER(vlbm3_box), C.c_int, C.POINTER(C.c_int)])
vlbm3_save = _sig("vlbm3_save", _st, [_P, C.c_void_p, C.POINTER(C.c_size_t)])
vlbm3_load = _sig("vlbm3_load", _st, [_P, C.c_void_p, C.c_size_t])
vlbm3_bind_allocator = _sig("vlbm3_bind_allocator", _st, [_P, _v.ALLOC_FN, _v.FREE_FN, C.c_void_p])

EXPORTED = ["vlbm3_create", "vlbm3_destroy", "vlbm3_footprint_bytes", "vlbm3_set_hierarchy",
            "vlbm3_regrid",
            "vlbm3_set_state", "vlbm3_set_populations", "vlbm3_get_state",
            "vlbm3_get_populations", "vlbm3_advance", "vlbm3_conserved_totals",
            "vlbm3_set_tuning", "vlbm3_set_profiling", "vlbm3_kernel_times",
            "vlbm3_active_cells", "vlbm3_sync", "vlbm3_tag", "vlbm3_tag_and_regrid", "vlbm3_get_boxes",
            "vlbm3_save", "vlbm3_load", "vlbm3_bind_allocator"]


def make_params(nx0, ny0, nz0, dx0, gamma=1.4, c=1.0, beta=0.9, r=2, max_levels=2,
                bc=(PERIODIC,) * 6, precision=FP64):
    p = vlbm3_params()
    p.nx0, p.ny0, p.nz0, p.dx0 = nx0, ny0, nz0, dx0
    for i in range(6):
        p.bc[i] = bc[i]
    p.gamma, p.c, p.beta, p.r, p.max_levels = gamma, c, beta, r, max_levels
    p.precision = precision
    return p


def make_boxes(boxes: Iterable[Sequence[int]]):
    boxes = list(boxes)
    arr = (vlbm3_box * max(1, len(boxes)))()
    for i, b in enumerate(boxes):
        arr[i] = vlbm3_box(*[int(v) for v in b])
    return arr, len(boxes)


def _dp(a):
    assert a.dtype == np.float64 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(_D)


class Solver3:
    """One 3-D hierarchy on one GPU. Arrays are (comp, z, y, x).

    memory="torch" (default when torch is importable) takes every device block
    from PyTorch's caching allocator on the solver's stream
    (vlbm3_bind_allocator); memory="library" lets the library hipMalloc."""

    def __init__(self, nx0, ny0, nz0, dx0, gamma=1.4, c=1.0, beta=0.9, r=2, max_levels=2,
                 bc=(PERIODIC,) * 6, stream=None, precision=FP64, memory="torch"):
        self.r, self.n0 = r, (nx0, ny0, nz0)
        self.p = make_params(nx0, ny0, nz0, dx0, gamma, c, beta, r, max_levels, bc, precision)
        self._h = C.c_void_p()
        self._alloc = None
        check(vlbm3_create(C.byref(self.p), _v._stream_handle(stream), C.byref(self._h)))
        if memory == "torch" and _v.torch is not None:
            self._alloc = _v.TorchAllocator(stream)
            check(vlbm3_bind_allocator(self._h, self._alloc.alloc_cb, self._alloc.free_cb, None))
        elif memory not in ("torch", "library"):
            raise ValueError(f"memory={memory!r}")

    @property
    def memory(self):
        return "torch" if self._alloc is not None else "library"

    @classmethod
    def from_case(cls, case, stream=None, max_levels=None, precision=FP64, memory="torch"):
        s = cls(case.nx0, case.ny0, case.nz0, case.dx0, case.gamma, case.c, case.beta, case.r,
                max_levels or case.nlev, case.bc, stream, precision, memory)
        s.set_hierarchy(case.boxes)
        for l, U in enumerate(case.states):
            if U is not None:
                s.set_state(l, U, lo=case.origin(l))
        return s

    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            vlbm3_destroy(self._h)
            self._h = C.c_void_p()
        self._alloc = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def shape(self, level):
        s = self.r ** level
        return self.n0[2] * s, self.n0[1] * s, self.n0[0] * s

    def set_hierarchy(self, boxes):
        arr, n = make_boxes(boxes)
        check(vlbm3_set_hierarchy(self._h, arr, n))

    def regrid(self, boxes):
        arr, n = make_boxes(boxes)
        check(vlbm3_regrid(self._h, arr, n))

    def _rect(self, level, lo, ext):
        NZ, NY, NX = self.shape(level)
        i0, j0, k0 = lo
        if ext is None:
            ext = (NX - i0, NY - j0, NZ - k0)
        return (i0, j0, k0), tuple(ext)

    def set_state(self, level, U, lo=(0, 0, 0)):
        U = np.ascontiguousarray(U, dtype=np.float64)
        nz, ny, nx = U.shape[1:]
        check(vlbm3_set_state(self._h, level, *lo, nx, ny, nz, _dp(U)))

    def set_populations(self, level, F, lo=(0, 0, 0)):
        F = np.ascontiguousarray(F, dtype=np.float64)
        nz, ny, nx = F.shape[1:]
        check(vlbm3_set_populations(self._h, level, *lo, nx, ny, nz, _dp(F)))

    def get_state(self, level, lo=(0, 0, 0), ext=None):
        lo, (nx, ny, nz) = self._rect(level, lo, ext)
        U = np.empty((5, nz, ny, nx))
        check(vlbm3_get_state(self._h, level, *lo, nx, ny, nz, _dp(U)))
        return U

    def get_populations(self, level, lo=(0, 0, 0), ext=None):
        lo, (nx, ny, nz) = self._rect(level, lo, ext)
        F = np.empty((30, nz, ny, nx))
        check(vlbm3_get_populations(self._h, level, *lo, nx, ny, nz, _dp(F)))
        return F

    def advance(self, n):
        check(vlbm3_advance(self._h, int(n)))

    def tag(self, level, threshold):
        """Density-gradient refinement tags of level `level` (uint8, Nz x Ny x Nx)."""
        t = np.zeros(self.shape(level), dtype=np.uint8)
        check(vlbm3_tag(self._h, int(level), float(threshold), t.ctypes.data_as(C.POINTER(C.c_uint8))))
        return t

    def tag_and_regrid(self, threshold, buffer=2, min_box=8, max_box=64):
        check(vlbm3_tag_and_regrid(self._h, float(threshold), int(buffer), int(min_box), int(max_box)))

    def save(self) -> bytes:
        n = C.c_size_t(0)
        check(vlbm3_save(self._h, None, C.byref(n)))
        buf = C.create_string_buffer(n.value)
        check(vlbm3_save(self._h, buf, C.byref(n)))
        return buf.raw[:n.value]

    def load(self, blob: bytes):
        buf = C.create_string_buffer(blob, len(blob))
        check(vlbm3_load(self._h, buf, len(blob)))

    def boxes(self):
        n = C.c_int()
        check(vlbm3_get_boxes(self._h, None, 0, C.byref(n)))
        arr = (vlbm3_box * max(1, n.value))()
        check(vlbm3_get_boxes(self._h, arr, n.value, C.byref(n)))
        return [(b.level, b.i0, b.j0, b.k0, b.nx, b.ny, b.nz) for b in arr[:n.value]]

    def totals(self):
        T, L = np.empty(5), np.empty(5)
        check(vlbm3_conserved_totals(self._h, _dp(T), _dp(L)))
        return T, L

    def set_tuning(self, tile_cells, flags=0):
        check(vlbm3_set_tuning(self._h, int(tile_cells), int(flags)))

    def set_profiling(self, enable=True):
        check(vlbm3_set_profiling(self._h, int(bool(enable))))

    def kernel_times(self):
        """{level: (total_ms, launches, cells)} since set_profiling(True)."""
        ms = (C.c_double * MAX_LEVELS)()
        calls = (C.c_long * MAX_LEVELS)()
        cells = (C.c_double * MAX_LEVELS)()
        check(vlbm3_kernel_times(self._h, ms, calls, cells))
        return {i: (ms[i], calls[i], cells[i]) for i in range(MAX_LEVELS) if calls[i]}

    def active_cells(self, level):
        return vlbm3_active_cells(self._h, int(level))

    def sync(self):
        check(vlbm3_sync(self._h))


def footprint_bytes(case, precision=FP64):
    p = make_params(case.nx0, case.ny0, case.nz0, case.dx0, case.gamma, case.c, case.beta,
                    case.r, case.nlev, case.bc, precision)
    arr, n = make_boxes(case.boxes)
    return vlbm3_footprint_bytes(C.byref(p), arr, n)
