"""Checkpoint and resume (vlbm_save / vlbm_load) through the C ABI.

A resumed run continues bit for bit: after regrids have grown the level
frames (row runs of the shear layer's two bands), and with the adaptive time
step (its clock travels in the checkpoint). Truncated or corrupted checkpoints,
and checkpoints that do not fit the context, are refused with VLBM_EINVAL."""
import ctypes as C
import struct

import numpy as np
import pytest

from paper_2609_35529_amd import vlbm
from paper_2609_35529_amd import workloads as wl
from tests.parity import gpu_solver

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True)
def _announce(request):
    print(f"\n[gpu] {request.node.name}", flush=True)
    yield


def _dynamic_kh(n0=64):
    case = wl.kelvin_helmholtz(n0=n0, seed=2, nlev=4, steps=0)
    return wl.Case(case.name, case.nx0, case.ny0, case.dx0, case.r, case.nlev, case.gamma, case.c,
                   case.beta, case.bc, [], [case.states[0]] + [None] * (case.nlev - 1), 0)


def _same_run(a, b, nlev):
    for l in range(nlev):
        assert np.array_equal(a.get_populations(l), b.get_populations(l), equal_nan=True), l
    Ta, La = a.totals()
    Tb, Lb = b.totals()
    assert np.array_equal(Ta, Tb) and np.array_equal(La, Lb)
    assert a.boxes() == b.boxes()


def test_resume_after_regrids_is_bitwise():
    """Three tag-and-regrid cycles grow the frames of levels 1-3 (two separate
    bands each); the checkpoint carries those frames, and the resumed run,
    with a regrid after the resume, equals the uninterrupted one."""
    case = _dynamic_kh()
    a = gpu_solver(case)
    for _ in range(3):
        a.tag_and_regrid(0.05, buffer=2, min_box=8, max_box=32)
        a.advance(3)
    assert max(b[0] for b in a.boxes()) == 3
    blob = a.save()
    a.advance(2)
    a.tag_and_regrid(0.05, buffer=2, min_box=8, max_box=32)
    a.advance(2)
    b = gpu_solver(case)
    b.load(blob)
    b.advance(2)
    b.tag_and_regrid(0.05, buffer=2, min_box=8, max_box=32)
    b.advance(2)
    _same_run(a, b, case.nlev)
    assert a.steps() == b.steps()


def test_resume_with_adaptive_time_step_is_bitwise():
    """The link speeds of the current and previous coarse step and the
    elapsed time travel in the checkpoint: the resumed run's populations and
    clock equal the uninterrupted run's, bit for bit."""
    case = wl.quadrant(n0=96, seed=1, steps=0)
    a = gpu_solver(case)
    a.set_time_stepping(True, 1.5)
    a.advance(3)
    blob = a.save()
    a.advance(4)
    b = gpu_solver(case)
    b.set_time_stepping(True, 1.5)
    b.advance(1)  # a context with its own, different clock
    b.load(blob)
    b.advance(4)
    _same_run(a, b, case.nlev)
    assert a.time() == b.time()


def _load_status(s, blob):
    buf = C.create_string_buffer(blob, len(blob))
    return vlbm.vlbm_load(s.handle, buf, len(blob))


def test_bad_checkpoints_are_refused():
    case = _dynamic_kh(32)
    a = gpu_solver(case)
    for _ in range(2):
        a.tag_and_regrid(0.05, buffer=2, min_box=8, max_box=32)
        a.advance(2)
    blob = a.save()
    b = gpu_solver(case)
    # truncated anywhere: header, boxes, frames, populations, slots
    for cut in (0, 10, 200, 260, 400, len(blob) // 3, len(blob) - 9, len(blob) - 1):
        assert _load_status(b, blob[:cut]) == vlbm.VLBM_EINVAL, cut
    # not a checkpoint
    assert _load_status(b, b"XXXXXXXX" + blob[8:]) == vlbm.VLBM_EINVAL
    # negative and oversized box counts (nboxes follows the magic and the params)
    off = 8 + C.sizeof(vlbm.vlbm_params)
    for n in (-1, 1 << 30):
        bad = blob[:off] + struct.pack("<i", n) + blob[off + 4:]
        assert _load_status(b, bad) == vlbm.VLBM_EINVAL, n
    # a context in another time stepping mode
    c = gpu_solver(case)
    c.set_time_stepping(True, 1.5)
    assert _load_status(c, blob) == vlbm.VLBM_EINVAL
    assert b"time step" in vlbm.vlbm_last_error()
    # the untouched checkpoint still loads and resumes
    assert _load_status(b, blob) == vlbm.VLBM_OK
    a.advance(2)
    b.advance(2)
    _same_run(a, b, case.nlev)
