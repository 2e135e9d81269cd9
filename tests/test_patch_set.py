"""The seeded uneven patch set (workloads.patch_set): counts and sizes in
their ranges, levels 1 and 2 in a 3:1 ratio of the drawn boxes, no two boxes
of a level overlapping, every level-2 box one level-1 cell inside a level-1
box, and the library's own host-side check accepting the hierarchy
(vlbm_footprint_bytes is 0 for an invalid one)."""
import numpy as np
import pytest

from paper_2609_35529_amd import vlbm
from paper_2609_35529_amd import workloads as wl


@pytest.mark.parametrize("seed", [0, 1, 7])
def test_patch_set_properties(seed):
    case = wl.patch_set(seed)
    b1 = [b for b in case.boxes if b[0] == 1]
    b2 = [b for b in case.boxes if b[0] == 2]
    drawn = int(case.name.split(" of ")[1].split()[0])
    assert 100 <= drawn <= 400
    assert len(b2) <= drawn // 4 and len(b1) <= drawn - drawn // 4
    assert len(b1) >= 0.8 * (drawn - drawn // 4) and len(b2) >= 0.5 * (drawn // 4)
    for lev, boxes in ((1, b1), (2, b2)):
        NY, NX = case.level_shape(lev)
        occ = np.zeros((NY, NX), dtype=np.int32)
        for (_, x, y, w, h) in boxes:
            assert 16 <= w <= 128 + 1 and 16 <= h <= 128 + 1
            assert x % 2 == 0 and y % 2 == 0 and w % 2 == 0 and h % 2 == 0
            assert 0 <= x and x + w <= NX and 0 <= y and y + h <= NY
            occ[y:y + h, x:x + w] += 1
        assert occ.max() <= 1
    for (_, x, y, w, h) in b2:
        fx, fy, fw, fh = x // 2, y // 2, w // 2, h // 2
        assert any(hx + 1 <= fx and fx + fw <= hx + hw - 1 and hy + 1 <= fy and fy + fh <= hy + hh - 1
                   for (_, hx, hy, hw, hh) in b1)
    assert vlbm.footprint_bytes(case) > 0
    assert wl.patch_set(seed).boxes == case.boxes  # deterministic
