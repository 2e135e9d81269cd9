"""ctypes binding of the C oracle (test infrastructure only).

Arrays follow the oracle's layout: populations ``F[16][ny][nx]`` with plane
index ``q*4+k`` (q: +x,-x,+y,-y; k: rho, rho u, rho v, rho E), conserved state
``U[4][ny][nx]``. Boxes are ``(level, i0, j0, nx, ny)`` in level-l cell indices.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

from . import build as _build

_lib = None

PERIODIC, OUTFLOW, REFLECT, INFLOW = 0, 1, 2, 3
EOS_IDEAL, EOS_STIFFENED, EOS_VDW = 0, 1, 2
MUT_NONE, MUT_REFLUX_END_LABEL, MUT_RECON_SIGMA_SIGN, MUT_REFLUX_LAST_ONLY = 0, 1, 2, 3
MUT_REGRID_RESTART_ALL, MUT_REGRID_NEW_FACE_HISTORY, MUT_WALL_NO_FLIP = 4, 5, 6
MUT_SENSOR_BOX_SUM, MUT_SENSOR_MAX_NORM, MUT_SLOPE_RATIO_INVERTED, MUT_TAG_ONE_SIDED = 7, 8, 9, 10
MUT_FLUX_SENSOR_RMS = 11
FMUT_NONE, FMUT_VDW_SIGN = 0, 1

_D = C.POINTER(C.c_double)
_I = C.POINTER(C.c_int)
_U8 = C.POINTER(C.c_uint8)


def lib():
    global _lib
    if _lib is None:
        path = _build.ensure_built()
        L = C.CDLL(path)
        L.orc_new.restype = C.c_void_p
        L.orc_new.argtypes = [C.c_int, C.c_int, C.c_double, C.c_int, C.c_int, C.c_double,
                              C.c_double, C.c_double, _I, _D]
        L.orc_free.argtypes = [C.c_void_p]
        L.orc_set_eos.argtypes = [C.c_void_p, C.c_int, C.c_double, C.c_double]
        L.orc_set_mutation.argtypes = [C.c_void_p, C.c_int]
        L.orc_set_function_mutation.argtypes = [C.c_int]
        L.orc_set_sensor.argtypes = [C.c_void_p, C.c_int, C.c_double, C.c_double, C.c_double]
        L.orc_get_beta.argtypes = [C.c_void_p, C.c_int, _D]
        L.orc_set_boxes.argtypes = [C.c_void_p, _I, C.c_int]
        L.orc_regrid.argtypes = [C.c_void_p, _I, C.c_int]
        for name in ("orc_set_state", "orc_get_state", "orc_get_pop", "orc_set_pop"):
            getattr(L, name).argtypes = [C.c_void_p, C.c_int, C.c_int, C.c_int, C.c_int, C.c_int,
                                         _D, C.c_long]
        L.orc_active_mask.argtypes = [C.c_void_p, C.c_int, _U8]
        L.orc_advance.argtypes = [C.c_void_p, C.c_int]
        L.orc_totals.argtypes = [C.c_void_p, _D, _D]
        L.orc_tag.argtypes = [C.c_void_p, C.c_int, C.c_double, _U8]
        L.orc_flux_sensor.argtypes = [C.c_void_p, C.c_int, _D]
        L.orc_tag_flux.argtypes = [C.c_void_p, C.c_int, C.c_double, _U8]
        L.orc_error.restype = C.c_char_p
        L.orc_feq.argtypes = [C.c_double, C.c_double, C.c_int, C.c_double, C.c_double, _D, _D]
        L.orc_flux.argtypes = [C.c_double, C.c_int, C.c_double, C.c_double, _D, _D, _D]
        L.orc_collide.argtypes = [C.c_double, C.c_double, C.c_double, C.c_int, C.c_double,
                                  C.c_double, _D, _D]
        L.orc_minmod.restype = C.c_double
        L.orc_minmod.argtypes = [C.c_double, C.c_double]
        L.orc_recon_value.restype = C.c_double
        L.orc_recon_value.argtypes = [C.c_double, C.c_double, C.c_double, C.c_int, C.c_int, C.c_int]
        L.orc_recon_value_scaled.restype = C.c_double
        L.orc_recon_value_scaled.argtypes = [C.c_double, C.c_double, C.c_double, C.c_int, C.c_int,
                                             C.c_int, C.c_double]
        L.orc_set_time_stepping.argtypes = [C.c_void_p, C.c_int, C.c_double]
        L.orc_time.restype = C.c_double
        L.orc_time.argtypes = [C.c_void_p]
        L.orc_link_speed.restype = C.c_double
        L.orc_link_speed.argtypes = [C.c_void_p]
        L.orc_split_block.argtypes = [C.c_int, _D, _D]
        L.orc_merge_block.restype = C.c_double
        L.orc_merge_block.argtypes = [C.c_int, _D]
        _lib = L
    return _lib


def _dp(a):
    return a.ctypes.data_as(_D)


def _check(rc):
    if rc != 0:
        raise RuntimeError("oracle: " + lib().orc_error().decode())


# ---------------------------------------------------------------- single ops
def feq(W, gamma, c, eos=EOS_IDEAL, a=0.0, b=0.0):
    W = np.ascontiguousarray(W, dtype=np.float64)
    out = np.empty(16)
    lib().orc_feq(gamma, c, eos, a, b, _dp(W), _dp(out))
    return out.reshape(4, 4)


def flux(W, gamma, eos=EOS_IDEAL, a=0.0, b=0.0):
    W = np.ascontiguousarray(W, dtype=np.float64)
    qx, qy = np.empty(4), np.empty(4)
    lib().orc_flux(gamma, eos, a, b, _dp(W), _dp(qx), _dp(qy))
    return qx, qy


def collide(g, gamma, c, beta, eos=EOS_IDEAL, a=0.0, b=0.0):
    g = np.ascontiguousarray(g, dtype=np.float64).reshape(16)
    out = np.empty(16)
    lib().orc_collide(gamma, c, beta, eos, a, b, _dp(g), _dp(out))
    return out.reshape(4, 4)


def set_function_mutation(mut):
    """Plant (mut != 0) or remove a mistake in the single-operation functions."""
    lib().orc_set_function_mutation(mut)


def minmod(a, b):
    return lib().orc_minmod(a, b)


def recon_value(out, prev, sigma, r, k, j):
    return lib().orc_recon_value(out, prev, sigma, r, k, j)


def split_block(r, fc):
    fc = np.ascontiguousarray(fc, dtype=np.float64).reshape(3, 3)
    ch = np.empty(r * r)
    lib().orc_split_block(r, _dp(fc), _dp(ch))
    return ch.reshape(r, r)


def merge_block(r, children):
    ch = np.ascontiguousarray(children, dtype=np.float64).reshape(r * r)
    return lib().orc_merge_block(r, _dp(ch))


# ---------------------------------------------------------------- solver
class Oracle:
    """A hierarchy of dense per-level grids advanced by the plain FP64 method."""

    def __init__(self, nx0, ny0, dx0, r=2, nlev=2, gamma=1.4, c=1.0, beta=0.9,
                 bc=(PERIODIC,) * 4, w_inflow=None, eos=EOS_IDEAL, eos_a=0.0, eos_b=0.0):
        self.nx0, self.ny0, self.dx0, self.r, self.nlev = nx0, ny0, dx0, r, nlev
        bc_a = (C.c_int * 4)(*bc)
        win = np.zeros(16) if w_inflow is None else np.ascontiguousarray(w_inflow, dtype=np.float64).reshape(16)
        self._h = lib().orc_new(nx0, ny0, dx0, r, nlev, gamma, c, beta, bc_a, _dp(win))
        if not self._h:
            raise RuntimeError("oracle: " + lib().orc_error().decode())
        if eos != EOS_IDEAL:
            lib().orc_set_eos(self._h, eos, eos_a, eos_b)

    def set_sensor(self, on=True, c_sensor=1.0, beta_min=0.5, beta_max=0.9):
        """Space/time-adaptive relaxation (eq. sensor-B), from the next step on."""
        if lib().orc_set_sensor(self._h, int(bool(on)), c_sensor, beta_min, beta_max):
            raise RuntimeError("oracle: " + lib().orc_error().decode())

    def set_time_stepping(self, on=True, kappa=1.5):
        """Adaptive time step: c per coarse step from the current state."""
        if lib().orc_set_time_stepping(self._h, int(bool(on)), kappa):
            raise RuntimeError("oracle: " + lib().orc_error().decode())

    def time(self):
        return lib().orc_time(self._h)

    def link_speed(self):
        return lib().orc_link_speed(self._h)

    def get_beta(self, level):
        """beta of every cell of `level` at its last step, (Ny, Nx); 0 where inactive."""
        out = np.zeros(self.shape(level))
        lib().orc_get_beta(self._h, level, _dp(out))
        return out

    def __del__(self):
        if getattr(self, "_h", None):
            lib().orc_free(self._h)
            self._h = None

    def shape(self, level):
        s = self.r ** level
        return self.ny0 * s, self.nx0 * s

    def set_mutation(self, mut):
        lib().orc_set_mutation(self._h, mut)

    @staticmethod
    def _boxes(boxes):
        arr = np.ascontiguousarray(np.asarray(boxes, dtype=np.int32).reshape(-1, 5))
        return arr, len(arr)

    def set_boxes(self, boxes):
        arr, n = self._boxes(boxes)
        _check(lib().orc_set_boxes(self._h, arr.ctypes.data_as(_I), n))

    def regrid(self, boxes):
        arr, n = self._boxes(boxes)
        _check(lib().orc_regrid(self._h, arr.ctypes.data_as(_I), n))

    def set_state(self, level, U, i0=0, j0=0):
        U = np.ascontiguousarray(U, dtype=np.float64)
        _, ny, nx = U.shape
        _check(lib().orc_set_state(self._h, level, i0, j0, nx, ny, _dp(U), nx))

    def set_pop(self, level, F, i0=0, j0=0):
        F = np.ascontiguousarray(F, dtype=np.float64)
        _, ny, nx = F.shape
        _check(lib().orc_set_pop(self._h, level, i0, j0, nx, ny, _dp(F), nx))

    def get_state(self, level, i0=0, j0=0, nx=None, ny=None):
        NY, NX = self.shape(level)
        nx = NX - i0 if nx is None else nx
        ny = NY - j0 if ny is None else ny
        U = np.empty((4, ny, nx))
        _check(lib().orc_get_state(self._h, level, i0, j0, nx, ny, _dp(U), nx))
        return U

    def get_pop(self, level, i0=0, j0=0, nx=None, ny=None):
        NY, NX = self.shape(level)
        nx = NX - i0 if nx is None else nx
        ny = NY - j0 if ny is None else ny
        F = np.empty((16, ny, nx))
        _check(lib().orc_get_pop(self._h, level, i0, j0, nx, ny, _dp(F), nx))
        return F

    def active_mask(self, level):
        NY, NX = self.shape(level)
        m = np.empty((NY, NX), dtype=np.uint8)
        _check(lib().orc_active_mask(self._h, level, m.ctypes.data_as(_U8)))
        return m.astype(bool)

    def advance(self, n):
        _check(lib().orc_advance(self._h, n))

    def totals(self):
        T, Lg = np.empty(4), np.empty(4)
        lib().orc_totals(self._h, _dp(T), _dp(Lg))
        return T, Lg

    def tag(self, level, thr):
        NY, NX = self.shape(level)
        t = np.empty((NY, NX), dtype=np.uint8)
        _check(lib().orc_tag(self._h, level, thr, t.ctypes.data_as(_U8)))
        return t

    def flux_sensor(self, level):
        """eq. amr-sigma: s = max_k |s_k| per active cell, (Ny, Nx), 0 elsewhere."""
        out = np.zeros(self.shape(level))
        _check(lib().orc_flux_sensor(self._h, level, _dp(out)))
        return out

    def tag_flux(self, level, thr):
        NY, NX = self.shape(level)
        t = np.empty((NY, NX), dtype=np.uint8)
        _check(lib().orc_tag_flux(self._h, level, thr, t.ctypes.data_as(_U8)))
        return t
