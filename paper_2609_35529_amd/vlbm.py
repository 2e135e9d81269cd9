"""Python binding of ``libvlbm.so`` (the C ABI of ``include/vlbm.h``).

Argument marshalling only: every step of the method runs in the HIP kernels of
the library. Importing this module loads the library and raises ``ImportError``
when it has not been built (``python -m paper_2609_35529_amd.build``); nothing
falls back to a CPU path. PyTorch, when used, only supplies device memory
(``bind_pool``) and the HIP stream the library launches on.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Iterable, Optional, Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libvlbm.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"libvlbm.so is not built ({LIB_PATH}); run `python -m paper_2609_35529_amd.build`")

# One HIP runtime per process: PyTorch ships its own libamdhip64 (same SONAME as
# the system one). Loading torch first makes libvlbm bind to that already-loaded
# runtime, so the streams torch hands over are streams of the runtime that
# launches the kernels; loading libvlbm first would put two runtimes in the
# process.
try:
    import torch  # noqa: F401
except ImportError:
    torch = None

_lib = C.CDLL(LIB_PATH)

VLBM_OK, VLBM_EINVAL, VLBM_ENOMEM, VLBM_ENEST, VLBM_EUNSTABLE, VLBM_EDEVICE, VLBM_ESTATE = (
    0, -1, -2, -3, -4, -5, -6)
PERIODIC, OUTFLOW, REFLECT, INFLOW = 0, 1, 2, 3
FP64, FP32, FP32_STORAGE = 0, 1, 2
EOS_IDEAL, EOS_STIFFENED, EOS_VDW = 0, 1, 2
# vlbm_set_tuning flags
TUNE_NT_STORES, TUNE_TWO_CELLS, TUNE_XCD_ORDER, TUNE_FUSE2 = 1, 2, 4, 16
TUNE_XCD_FUSED, TUNE_GRAPHS, TUNE_SMALL_TILES = 512, 1024, 2048


class vlbm_params(C.Structure):
    _fields_ = [("nx0", C.c_int), ("ny0", C.c_int), ("dx0", C.c_double), ("bc", C.c_int * 4),
                ("w_inflow", (C.c_double * 4) * 4), ("gamma", C.c_double), ("c", C.c_double),
                ("beta", C.c_double), ("r", C.c_int), ("max_levels", C.c_int),
                ("precision", C.c_int), ("eos", C.c_int), ("eos_a", C.c_double),
                ("eos_b", C.c_double)]


class vlbm_box(C.Structure):
    _fields_ = [("level", C.c_int), ("i0", C.c_int), ("j0", C.c_int), ("nx", C.c_int),
                ("ny", C.c_int)]


_P = C.c_void_p
_D = C.POINTER(C.c_double)
_st = C.c_int


def _sig(name, res, args):
    f = getattr(_lib, name)
    f.restype = res
    f.argtypes = args
    return f


vlbm_create = _sig("vlbm_create", _st, [C.POINTER(vlbm_params), _P, C.POINTER(_P)])
vlbm_destroy = _sig("vlbm_destroy", None, [_P])
vlbm_bind_pool = _sig("vlbm_bind_pool", _st, [_P, _P, C.c_size_t])
ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p)
FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p)
vlbm_bind_allocator = _sig("vlbm_bind_allocator", _st, [_P, ALLOC_FN, FREE_FN, _P])
vlbm_footprint_bytes = _sig("vlbm_footprint_bytes", C.c_size_t,
                            [C.POINTER(vlbm_params), C.POINTER(vlbm_box), C.c_int])
vlbm_set_hierarchy = _sig("vlbm_set_hierarchy", _st, [_P, C.POINTER(vlbm_box), C.c_int])
_rect = [_P, C.c_int, C.c_int, C.c_int, C.c_int, C.c_int, _D, C.c_long]
vlbm_set_state = _sig("vlbm_set_state", _st, _rect)
vlbm_set_populations = _sig("vlbm_set_populations", _st, _rect)
vlbm_get_state = _sig("vlbm_get_state", _st, _rect)
vlbm_get_state_noalloc = _sig("vlbm_get_state_noalloc", _st, _rect)
vlbm_get_populations = _sig("vlbm_get_populations", _st, _rect)
vlbm_advance = _sig("vlbm_advance", _st, [_P, C.c_int])
vlbm_conserved_totals = _sig("vlbm_conserved_totals", _st, [_P, _D, _D])
vlbm_regrid = _sig("vlbm_regrid", _st, [_P, C.POINTER(vlbm_box), C.c_int])
vlbm_tag = _sig("vlbm_tag", _st, [_P, C.c_int, C.c_double, C.POINTER(C.c_uint8)])
vlbm_set_tag_indicator = _sig("vlbm_set_tag_indicator", _st, [_P, C.c_int])
TAG_DENSITY, TAG_FLUX = 0, 1
vlbm_tag_and_regrid = _sig("vlbm_tag_and_regrid", _st,
                           [_P, C.c_double, C.c_int, C.c_int, C.c_int])
vlbm_get_boxes = _sig("vlbm_get_boxes", _st, [_P, C.POINTER(vlbm_box), C.c_int,
                                                  C.POINTER(C.c_int)])
vlbm_check_health = _sig("vlbm_check_health", _st, [_P])
vlbm_save = _sig("vlbm_save", _st, [_P, _P, C.POINTER(C.c_size_t)])
vlbm_load = _sig("vlbm_load", _st, [_P, _P, C.c_size_t])
vlbm_batch_advance = _sig("vlbm_batch_advance", _st, [C.POINTER(_P), C.POINTER(C.c_int), C.c_int])
vlbm_set_tuning = _sig("vlbm_set_tuning", _st, [_P, C.c_int, C.c_int])
vlbm_autotune = _sig("vlbm_autotune", _st, [_P, C.c_int, C.POINTER(C.c_int), C.POINTER(C.c_int)])
vlbm_steps = _sig("vlbm_steps", C.c_long, [_P])
vlbm_active_cells = _sig("vlbm_active_cells", C.c_long, [_P, C.c_int])
vlbm_sync = _sig("vlbm_sync", _st, [_P])
vlbm_set_profiling = _sig("vlbm_set_profiling", _st, [_P, C.c_int])
vlbm_kernel_times = _sig("vlbm_kernel_times", _st, [_P, _D, C.POINTER(C.c_long), _D])
vlbm_set_sensor = _sig("vlbm_set_sensor", _st, [_P, C.c_int, C.c_double, C.c_double, C.c_double])
vlbm_get_beta = _sig("vlbm_get_beta", _st, _rect)
vlbm_set_time_stepping = _sig("vlbm_set_time_stepping", _st, [_P, C.c_int, C.c_double])
vlbm_time = _sig("vlbm_time", _st, [_P, _D, _D])
MAX_LEVELS = 8
vlbm_last_error = _sig("vlbm_last_error", C.c_char_p, [])

EXPORTED = ["vlbm_create", "vlbm_destroy", "vlbm_bind_pool", "vlbm_footprint_bytes",
            "vlbm_set_hierarchy", "vlbm_set_state", "vlbm_set_populations", "vlbm_advance",
            "vlbm_get_state", "vlbm_get_populations", "vlbm_conserved_totals", "vlbm_regrid",
            "vlbm_tag", "vlbm_tag_and_regrid", "vlbm_get_boxes", "vlbm_check_health",
            "vlbm_save", "vlbm_load", "vlbm_batch_advance", "vlbm_set_tuning", "vlbm_autotune",
            "vlbm_steps", "vlbm_active_cells", "vlbm_sync", "vlbm_last_error",
            "vlbm_set_profiling", "vlbm_kernel_times", "vlbm_set_sensor", "vlbm_get_beta",
            "vlbm_set_time_stepping", "vlbm_time", "vlbm_get_state_noalloc", "vlbm_bind_allocator", "vlbm_set_tag_indicator"]


class VLBMError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"vlbm status {status}: {msg}")
        self.status = status


def check(status):
    if status != VLBM_OK:
        raise VLBMError(status, vlbm_last_error().decode())
    return status


def make_params(nx0, ny0, dx0, gamma, c, beta, r=2, max_levels=2, bc=(PERIODIC,) * 4,
                w_inflow=None, precision=FP64, eos=None) -> vlbm_params:
    """eos: None (ideal gas) or (kind, a, b) with kind one of EOS_*."""
    p = vlbm_params()
    p.nx0, p.ny0, p.dx0 = nx0, ny0, dx0
    for s in range(4):
        p.bc[s] = int(bc[s])
    if w_inflow is not None:
        w = np.asarray(w_inflow, dtype=np.float64).reshape(4, 4)
        for s in range(4):
            for k in range(4):
                p.w_inflow[s][k] = float(w[s, k])
    p.gamma, p.c, p.beta = gamma, c, beta
    p.r, p.max_levels, p.precision = r, max_levels, precision
    if eos is not None:
        p.eos, p.eos_a, p.eos_b = int(eos[0]), float(eos[1]), float(eos[2])
    return p


def make_boxes(boxes: Iterable[Sequence[int]]):
    boxes = list(boxes)
    arr = (vlbm_box * max(1, len(boxes)))()
    for i, b in enumerate(boxes):
        arr[i].level, arr[i].i0, arr[i].j0, arr[i].nx, arr[i].ny = (int(v) for v in b)
    return arr, len(boxes)


def _dp(a):
    return a.ctypes.data_as(_D)


def _stream_handle(stream):
    if stream is None:
        return None
    if isinstance(stream, int):
        return C.c_void_p(stream)
    return C.c_void_p(int(stream.cuda_stream))


class TorchAllocator:
    """Device blocks for the library from PyTorch's caching allocator, on the
    library's stream (blocks freed there are reused in that stream's order).
    Holds each block's tensor until the library releases it."""

    def __init__(self, stream=None):
        if torch is None:
            raise ImportError("torch is needed for the PyTorch allocator")
        self.stream = stream
        self.live = {}
        self.bytes_in_use = 0
        self.alloc_cb = ALLOC_FN(self._alloc)
        self.free_cb = FREE_FN(self._free)

    def _alloc(self, nbytes, user):
        try:
            ctx = torch.cuda.stream(self.stream) if self.stream is not None else None
            if ctx is not None:
                with ctx:
                    t = torch.empty(int(nbytes), dtype=torch.uint8, device="cuda")
            else:
                t = torch.empty(int(nbytes), dtype=torch.uint8, device="cuda")
        except Exception:  # out of memory: the library reports VLBM_ENOMEM
            return None
        p = t.data_ptr()
        self.live[p] = t
        self.bytes_in_use += int(nbytes)
        return p

    def _free(self, ptr, user):
        t = self.live.pop(ptr, None)
        if t is not None:
            self.bytes_in_use -= t.numel()


def torch_pool(nbytes, device="cuda"):
    """A device tensor of nbytes bytes from PyTorch's allocator, to bind as a
    context's memory pool (vlbm_bind_pool)."""
    if torch is None:
        raise ImportError("torch is needed to allocate a device pool")
    return torch.empty(int(nbytes), dtype=torch.uint8, device=device)


class Solver:
    """One VLBM hierarchy living on the GPU (a ``vlbm_ctx``).

    Device memory (PyTorch is the allocator unless memory="library"):
    memory="torch" (default when torch is importable) takes every block from
    PyTorch's caching allocator on the solver's stream (vlbm_bind_allocator);
    `pool` is one device tensor the library suballocates (vlbm_bind_pool), and
    `pool_bytes` asks for such a tensor of that size."""

    def __init__(self, nx0, ny0, dx0, gamma=1.4, c=1.0, beta=0.9, r=2, max_levels=2,
                 bc=(PERIODIC,) * 4, w_inflow=None, precision=FP64, stream=None, pool=None,
                 eos=None, pool_bytes=None, memory="torch"):
        self.params = make_params(nx0, ny0, dx0, gamma, c, beta, r, max_levels, bc, w_inflow,
                                  precision, eos)
        self.nx0, self.ny0, self.r = nx0, ny0, r
        self.max_levels = max_levels
        self._h = C.c_void_p()
        self._pool = None
        self._alloc = None
        check(vlbm_create(C.byref(self.params), _stream_handle(stream), C.byref(self._h)))
        if pool is None and pool_bytes:
            pool = torch_pool(pool_bytes)
        if pool is not None:
            self._pool = pool  # keeps the device tensor alive as long as the context
            check(vlbm_bind_pool(self._h, C.c_void_p(pool.data_ptr()),
                                 pool.numel() * pool.element_size()))
        elif memory == "torch" and torch is not None:
            self._alloc = TorchAllocator(stream)
            check(vlbm_bind_allocator(self._h, self._alloc.alloc_cb, self._alloc.free_cb, None))
        elif memory not in ("torch", "library"):
            raise ValueError(f"memory={memory!r}")

    @property
    def memory(self):
        return "pool" if self._pool is not None else "torch" if self._alloc is not None else "library"

    @classmethod
    def from_case(cls, case, precision=FP64, stream=None, pool=None, max_levels=None, pool_bytes=None,
                  memory="torch"):
        s = cls(case.nx0, case.ny0, case.dx0, case.gamma, case.c, case.beta, case.r,
                max_levels or case.nlev, case.bc, case.w_inflow, precision, stream, pool,
                eos=getattr(case, "eos", None), pool_bytes=pool_bytes, memory=memory)
        s.set_hierarchy(case.boxes)
        for l in range(case.nlev):
            if case.states[l] is not None:
                s.set_state(l, case.states[l])
        return s

    @property
    def handle(self):
        return self._h

    def close(self):
        if self._h:
            vlbm_destroy(self._h)
            self._h = C.c_void_p()
        self._pool = None
        self._alloc = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def shape(self, level):
        s = self.r ** level
        return self.ny0 * s, self.nx0 * s

    def set_hierarchy(self, boxes):
        arr, n = make_boxes(boxes)
        check(vlbm_set_hierarchy(self._h, arr, n))

    def regrid(self, boxes):
        arr, n = make_boxes(boxes)
        check(vlbm_regrid(self._h, arr, n))

    def set_tag_indicator(self, kind):
        """TAG_DENSITY (density gradient) or TAG_FLUX (eq. amr-sigma)."""
        check(vlbm_set_tag_indicator(self._h, int(kind)))

    def tag_and_regrid(self, threshold, buffer=4, min_box=16, max_box=128):
        check(vlbm_tag_and_regrid(self._h, threshold, buffer, min_box, max_box))

    def boxes(self):
        n = C.c_int()
        check(vlbm_get_boxes(self._h, None, 0, C.byref(n)))
        arr = (vlbm_box * max(1, n.value))()
        check(vlbm_get_boxes(self._h, arr, n.value, C.byref(n)))
        return [(b.level, b.i0, b.j0, b.nx, b.ny) for b in arr[:n.value]]

    def set_state(self, level, U, i0=0, j0=0):
        U = np.ascontiguousarray(U, dtype=np.float64)
        _, ny, nx = U.shape
        check(vlbm_set_state(self._h, level, i0, j0, nx, ny, _dp(U), nx))

    def set_populations(self, level, F, i0=0, j0=0):
        F = np.ascontiguousarray(F, dtype=np.float64)
        _, ny, nx = F.shape
        check(vlbm_set_populations(self._h, level, i0, j0, nx, ny, _dp(F), nx))

    def _rect(self, level, i0, j0, nx, ny):
        NY, NX = self.shape(level)
        return (NX - i0 if nx is None else nx), (NY - j0 if ny is None else ny)

    def get_state(self, level, i0=0, j0=0, nx=None, ny=None):
        nx, ny = self._rect(level, i0, j0, nx, ny)
        U = np.empty((4, ny, nx))
        check(vlbm_get_state(self._h, level, i0, j0, nx, ny, _dp(U), nx))
        return U

    def get_state_noalloc(self, level, i0=0, j0=0, nx=None, ny=None, out=None):
        """As get_state, through the allocation-free entry point (static
        per-GPU staging; at most 1 Mi cells of the rectangle inside the frame)."""
        nx, ny = self._rect(level, i0, j0, nx, ny)
        U = np.empty((4, ny, nx)) if out is None else out
        check(vlbm_get_state_noalloc(self._h, level, i0, j0, nx, ny, _dp(U), U.shape[2]))
        return U

    def get_populations(self, level, i0=0, j0=0, nx=None, ny=None):
        nx, ny = self._rect(level, i0, j0, nx, ny)
        F = np.empty((16, ny, nx))
        check(vlbm_get_populations(self._h, level, i0, j0, nx, ny, _dp(F), nx))
        return F

    def advance(self, n):
        check(vlbm_advance(self._h, int(n)))

    def totals(self):
        T, L = np.empty(4), np.empty(4)
        check(vlbm_conserved_totals(self._h, _dp(T), _dp(L)))
        return T, L

    def tag(self, level, threshold):
        NY, NX = self.shape(level)
        t = np.empty((NY, NX), dtype=np.uint8)
        check(vlbm_tag(self._h, level, threshold, t.ctypes.data_as(C.POINTER(C.c_uint8))))
        return t

    def check_health(self):
        return vlbm_check_health(self._h) == VLBM_OK

    def save(self) -> bytes:
        n = C.c_size_t()
        check(vlbm_save(self._h, None, C.byref(n)))
        buf = C.create_string_buffer(n.value)
        check(vlbm_save(self._h, buf, C.byref(n)))
        return buf.raw[:n.value]

    def load(self, blob: bytes):
        buf = C.create_string_buffer(blob, len(blob))
        check(vlbm_load(self._h, buf, len(blob)))

    def steps(self):
        return vlbm_steps(self._h)

    def active_cells(self, level):
        return vlbm_active_cells(self._h, int(level))

    def set_profiling(self, enable=True):
        check(vlbm_set_profiling(self._h, int(bool(enable))))

    def kernel_times(self):
        """{(level, fused): (total_ms, launches, cells)} for the launches
        recorded since set_profiling(True); cells: active cells advanced, summed
        over the launches."""
        ms = (C.c_double * (2 * MAX_LEVELS))()
        calls = (C.c_long * (2 * MAX_LEVELS))()
        cells = (C.c_double * (2 * MAX_LEVELS))()
        check(vlbm_kernel_times(self._h, ms, calls, cells))
        return {(i // 2, bool(i % 2)): (ms[i], calls[i], cells[i])
                for i in range(2 * MAX_LEVELS) if calls[i]}

    def set_sensor(self, on=True, c_sensor=1.0, beta_min=0.5, beta_max=0.9):
        """Space/time-adaptive relaxation parameter (Sec. 2.2, eq. sensor-B)."""
        check(vlbm_set_sensor(self._h, int(bool(on)), float(c_sensor), float(beta_min),
                              float(beta_max)))

    def get_beta(self, level, i0=0, j0=0, nx=None, ny=None):
        """beta of the level's latest step per active cell (NaN elsewhere)."""
        nx, ny = self._rect(level, i0, j0, nx, ny)
        b = np.empty((ny, nx))
        check(vlbm_get_beta(self._h, level, i0, j0, nx, ny, _dp(b), nx))
        return b

    def set_time_stepping(self, on=True, kappa=1.5):
        """Adaptive time step: c chosen every coarse step from the state."""
        check(vlbm_set_time_stepping(self._h, int(bool(on)), float(kappa)))

    def time(self):
        """(elapsed time, link speed of the last coarse step)."""
        t, c = C.c_double(), C.c_double()
        check(vlbm_time(self._h, C.byref(t), C.byref(c)))
        return t.value, c.value

    def set_tuning(self, tile_cells, flags=0):
        check(vlbm_set_tuning(self._h, int(tile_cells), int(flags)))

    def autotune(self, steps_per_trial=5):
        t, f = C.c_int(), C.c_int()
        check(vlbm_autotune(self._h, int(steps_per_trial), C.byref(t), C.byref(f)))
        return t.value, f.value

    def sync(self):
        check(vlbm_sync(self._h))


def batch_advance(solvers, n_steps):
    arr = (C.c_void_p * len(solvers))(*[s.handle.value for s in solvers])
    ns = (C.c_int * len(solvers))(*[int(n) for n in n_steps])
    check(vlbm_batch_advance(arr, ns, len(solvers)))


def footprint_bytes(case, precision=FP64, max_levels=None):
    p = make_params(case.nx0, case.ny0, case.dx0, case.gamma, case.c, case.beta, case.r,
                    max_levels or case.nlev, case.bc, case.w_inflow, precision,
                    getattr(case, "eos", None))
    arr, n = make_boxes(case.boxes)
    return vlbm_footprint_bytes(C.byref(p), arr, n)
