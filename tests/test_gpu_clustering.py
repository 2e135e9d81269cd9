"""Clustering of vlbm_tag_and_regrid against a reference written here from
its documented rule (include/vlbm.h, vlbm_tag_and_regrid), on the tags the
library reports (vlbm_tag, which is bit-exact with the oracle's tags):

  * a tagged cell also tags its parent, finest level first;
  * level l is cut into tiles of side T = ceil(min_box / r) cells; a tile is
    hit when a tagged cell lies within `buffer` cells of it (periodic sides
    wrapped, other sides clipped);
  * a hit tile is kept when it and the ring of cells around it are covered
    by the boxes just made for level l (level 0: everything; cells beyond a
    non-periodic side exempt);
  * kept tiles merge greedily: along a tile row into runs of at most
    maxT = max(1, max_box // (T r)) tiles, stacked while the run below is the
    same, up to maxT tile rows; each rectangle becomes a level-(l+1) box.

The box lists must be identical (as sets) after every regrid, on a periodic
shear layer with four levels, the shock-bubble (inflow, outflow, reflecting
sides) and a strip with mixed sides."""
import math

import numpy as np
import pytest

from paper_2609_35529_amd import workloads as wl
from tests.parity import gpu_solver

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True)
def _announce(request):
    print(f"\n[gpu] {request.node.name}", flush=True)
    yield


def _dilate(a, buf, perx, pery):
    out = a.copy()
    for axis, per in ((1, perx), (0, pery)):
        src = out.copy()
        for s in range(1, buf + 1):
            for sgn in (1, -1):
                if per:
                    out |= np.roll(src, sgn * s, axis=axis)
                else:
                    sh = np.zeros_like(src)
                    if axis == 1:
                        if sgn > 0:
                            sh[:, s:] = src[:, :-s]
                        else:
                            sh[:, :-s] = src[:, s:]
                    else:
                        if sgn > 0:
                            sh[s:, :] = src[:-s, :]
                        else:
                            sh[:-s, :] = src[s:, :]
                    out |= sh
    return out


def reference_boxes(tags, shapes, r, nlev_present, max_levels, perx, pery, buffer, min_box, max_box):
    tags = [t.astype(bool).copy() for t in tags]
    for l in range(nlev_present - 1, 0, -1):  # parents of tagged cells, finest first
        NY, NX = shapes[l - 1]
        ys, xs = np.nonzero(tags[l])
        tags[l - 1][ys // r, xs // r] = True
    T = max(1, math.ceil(min_box / r))
    maxT = max(1, max_box // (T * r))
    nclu = min(nlev_present, max_levels - 1)
    boxes = []
    cov = None  # None: everything covered
    for l in range(nclu):
        NY, NX = shapes[l]
        D = _dilate(tags[l], buffer, perx, pery)
        ntx, nty = -(-NX // T), -(-NY // T)

        def covered(x, y):
            if x < 0 or x >= NX:
                if not perx:
                    return True
                x %= NX
            if y < 0 or y >= NY:
                if not pery:
                    return True
                y %= NY
            return True if cov is None else bool(cov[y, x])

        def allowed(tx, ty):
            x0, y0 = tx * T, ty * T
            x1, y1 = min(NX, x0 + T), min(NY, y0 + T)
            for y in range(y0, y1):
                for x in range(x0 - 1, x1 + 1):
                    if not covered(x, y):
                        return False
            for y in (y0 - 1, y1):
                for x in range(x0, x1):
                    if not covered(x, y):
                        return False
            return True

        made = []
        opened = []  # [a, b, y0, h]
        for ty in range(nty):
            runs = []
            ra = rb = -1
            for tx in range(ntx):
                x0, y0 = tx * T, ty * T
                if not D[y0:min(NY, y0 + T), x0:min(NX, x0 + T)].any() or not allowed(tx, ty):
                    continue
                if ra >= 0 and tx == rb and rb - ra < maxT:
                    rb = tx + 1
                    continue
                if ra >= 0:
                    runs.append([ra, rb, ty, 1])
                ra, rb = tx, tx + 1
            if ra >= 0:
                runs.append([ra, rb, ty, 1])
            for o in opened:
                cont = False
                for n in runs:
                    if n[0] == o[0] and n[1] == o[1] and n[3] == 1 and o[3] < maxT:
                        n[2], n[3] = o[2], o[3] + 1
                        cont = True
                        break
                if not cont:
                    made.append(o)
            opened = runs
        made.extend(opened)
        lev = []
        for a, b, y0, h in made:
            x0, x1 = a * T, min(NX, b * T)
            ya, yb = y0 * T, min(NY, (y0 + h) * T)
            lev.append((l + 1, x0 * r, ya * r, (x1 - x0) * r, (yb - ya) * r))
        boxes.extend(lev)
        if not lev or l + 2 >= max_levels:
            break
        NYf, NXf = shapes[l + 1]
        cov = np.zeros((NYf, NXf), dtype=bool)
        for (_, i0, j0, nx, ny) in lev:
            cov[j0:j0 + ny, i0:i0 + nx] = True
    return sorted(boxes)


def _cases():
    kh = wl.kelvin_helmholtz(n0=64, seed=3, nlev=4, steps=0)
    kh = wl.Case(kh.name, kh.nx0, kh.ny0, kh.dx0, kh.r, kh.nlev, kh.gamma, kh.c, kh.beta, kh.bc, [],
                 [kh.states[0]] + [None] * (kh.nlev - 1), 0)
    sb = wl.shock_bubble(nx0=128, ny0=32, nlev=3, steps=0)
    sb = wl.Case(sb.name, sb.nx0, sb.ny0, sb.dx0, sb.r, sb.nlev, sb.gamma, sb.c, sb.beta, sb.bc, [],
                 sb.states, 0, w_inflow=sb.w_inflow)
    return {"kh64": (kh, (0.05, 2, 8, 32)), "kh64_wide": (kh, (0.02, 4, 16, 64)),
            "shock_bubble": (sb, (0.05, 2, 8, 32)), "shock_bubble_odd": (sb, (0.03, 3, 6, 24))}


@pytest.mark.parametrize("name", ["kh64", "kh64_wide", "shock_bubble", "shock_bubble_odd"])
def test_boxes_match_reference(name):
    case, (thr, buf, mn, mx) = _cases()[name]
    g = gpu_solver(case)
    perx, pery = case.bc[0] == wl.PERIODIC, case.bc[2] == wl.PERIODIC
    total = 0
    for cycle in range(4):
        nlev_present = 1 + max([b[0] for b in g.boxes()] + [0])
        shapes = [g.shape(l) for l in range(case.nlev)]
        tags = [g.tag(l, thr) for l in range(nlev_present)]
        ref = reference_boxes(tags, shapes, case.r, nlev_present, case.nlev, perx, pery, buf, mn, mx)
        g.tag_and_regrid(thr, buffer=buf, min_box=mn, max_box=mx)
        got = sorted(g.boxes())
        assert got == ref, (name, cycle, len(got), len(ref))
        total += len(got)
        g.advance(3)
    assert total > 0
