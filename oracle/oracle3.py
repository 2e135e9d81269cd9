"""ctypes binding of the 3-D (D3Q6) C oracle (test infrastructure only).

Arrays follow the oracle's layout: populations ``F[30][Nz][Ny][Nx]`` with
plane index ``q*5+k`` (q: +x,-x,+y,-y,+z,-z; k: rho, rho u, rho v, rho w,
rho E), conserved state ``U[5][Nz][Ny][Nx]``, whole levels. Boxes are
``(level, i0, j0, k0, nx, ny, nz)`` in level-l cell indices.
"""
from __future__ import annotations

import ctypes as C

import numpy as np

from . import oracle as _o2

PERIODIC, OUTFLOW, REFLECT = 0, 1, 2

_D = C.POINTER(C.c_double)
_I = C.POINTER(C.c_int)
_U8 = C.POINTER(C.c_uint8)
_ready = False


# planted mistakes (vlbm3_oracle.h)
(MUT_NONE, MUT_TAN_SLOPE_SIGN, MUT_TAN_OFFSETS_SWAPPED, MUT_REFLUX_R2, MUT_WALL_NO_FLIP,
 MUT_MERGE_R2, MUT_SPLIT_SLOPE_SIGN, MUT_REGRID_RESTART_ALL, MUT_REGRID_NEW_FACE_HISTORY) = range(9)


def lib():
    global _ready
    L = _o2.lib()
    if not _ready:
        L.orc3_new.restype = C.c_void_p
        L.orc3_new.argtypes = [C.c_int, C.c_int, C.c_int, C.c_double, C.c_int, C.c_int,
                               C.c_double, C.c_double, C.c_double, _I]
        L.orc3_free.argtypes = [C.c_void_p]
        L.orc3_set_mutation.argtypes = [C.c_void_p, C.c_int]
        L.orc3_set_boxes.argtypes = [C.c_void_p, _I, C.c_int]
        L.orc3_regrid.argtypes = [C.c_void_p, _I, C.c_int]
        L.orc3_tag.argtypes = [C.c_void_p, C.c_int, C.c_double, _U8]
        for name in ("orc3_set_state", "orc3_set_pop", "orc3_get_pop", "orc3_get_state"):
            getattr(L, name).argtypes = [C.c_void_p, C.c_int, _D]
        L.orc3_active_mask.argtypes = [C.c_void_p, C.c_int, _U8]
        L.orc3_advance.argtypes = [C.c_void_p, C.c_int]
        L.orc3_totals.argtypes = [C.c_void_p, _D, _D]
        L.orc3_shape.argtypes = [C.c_void_p, C.c_int, _I]
        L.orc3_error.restype = C.c_char_p
        L.orc3_flux.argtypes = [C.c_double, _D, _D, _D, _D]
        L.orc3_feq.argtypes = [C.c_double, C.c_double, _D, _D]
        L.orc3_collide.argtypes = [C.c_double, C.c_double, C.c_double, _D, _D]
        _ready = True
    return L


def _dp(a):
    assert a.dtype == np.float64 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(_D)


def flux(W, gamma=1.4):
    W = np.ascontiguousarray(W, dtype=np.float64)
    Q = np.zeros((3, 5))
    lib().orc3_flux(gamma, _dp(W), _dp(Q[0]), _dp(Q[1]), _dp(Q[2]))
    return Q


def feq(W, gamma=1.4, c=1.0):
    W = np.ascontiguousarray(W, dtype=np.float64)
    f = np.zeros(30)
    lib().orc3_feq(gamma, c, _dp(W), _dp(f))
    return f.reshape(6, 5)


def collide(g, gamma=1.4, c=1.0, beta=0.5):
    g = np.ascontiguousarray(np.asarray(g, dtype=np.float64).reshape(30))
    out = np.zeros(30)
    lib().orc3_collide(gamma, c, beta, _dp(g), _dp(out))
    return out.reshape(6, 5)


class Oracle3:
    """Three-dimensional counterpart of ``oracle.Oracle``."""

    def __init__(self, nx0, ny0, nz0, dx0, r=2, nlev=1, gamma=1.4, c=1.0, beta=0.9,
                 bc=(PERIODIC,) * 6):
        self.r, self.nlev = r, nlev
        b = (C.c_int * 6)(*bc)
        self._h = lib().orc3_new(nx0, ny0, nz0, dx0, r, nlev, gamma, c, beta, b)
        if not self._h:
            raise RuntimeError("oracle3: " + lib().orc3_error().decode())

    def __del__(self):
        if getattr(self, "_h", None):
            lib().orc3_free(self._h)
            self._h = None

    def set_mutation(self, mut):
        lib().orc3_set_mutation(self._h, mut)

    def shape(self, level):
        s = (C.c_int * 3)()
        lib().orc3_shape(self._h, level, s)
        return s[2], s[1], s[0]  # (Nz, Ny, Nx)

    def set_boxes(self, boxes):
        flat = [int(v) for b in boxes for v in b]
        arr = (C.c_int * max(1, len(flat)))(*flat)
        if lib().orc3_set_boxes(self._h, arr, len(boxes)):
            raise RuntimeError("oracle3: " + lib().orc3_error().decode())

    def regrid(self, boxes):
        flat = [int(v) for b in boxes for v in b]
        arr = (C.c_int * max(1, len(flat)))(*flat)
        if lib().orc3_regrid(self._h, arr, len(boxes)):
            raise RuntimeError("oracle3: " + lib().orc3_error().decode())

    def set_state(self, level, U):
        U = np.ascontiguousarray(U, dtype=np.float64)
        assert U.shape == (5,) + self.shape(level)
        lib().orc3_set_state(self._h, level, _dp(U))

    def set_pop(self, level, F):
        F = np.ascontiguousarray(F, dtype=np.float64)
        assert F.shape == (30,) + self.shape(level)
        lib().orc3_set_pop(self._h, level, _dp(F))

    def get_pop(self, level):
        F = np.empty((30,) + self.shape(level))
        lib().orc3_get_pop(self._h, level, _dp(F))
        return F

    def get_state(self, level):
        U = np.empty((5,) + self.shape(level))
        lib().orc3_get_state(self._h, level, _dp(U))
        return U

    def active_mask(self, level):
        m = np.empty(self.shape(level), dtype=np.uint8)
        lib().orc3_active_mask(self._h, level, m.ctypes.data_as(_U8))
        return m.astype(bool)

    def advance(self, n):
        lib().orc3_advance(self._h, int(n))

    def tag(self, level, thr):
        """Density-gradient refinement tags of the active cells (uint8, Nz x Ny x Nx)."""
        t = np.zeros(self.shape(level), dtype=np.uint8)
        if lib().orc3_tag(self._h, level, float(thr), t.ctypes.data_as(_U8)):
            raise RuntimeError("oracle3: bad level")
        return t

    def totals(self):
        T, L = np.zeros(5), np.zeros(5)
        lib().orc3_totals(self._h, _dp(T), _dp(L))
        return T, L
