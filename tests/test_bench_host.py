"""Host side of bench.py: the single-GPU refusal and the sizes of the timed
workloads (fine-equivalent and actual cell updates per coarse step)."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


@pytest.mark.parametrize("extra", [[], ["--workload", "blast3d"], ["--serve-only"]])
def test_more_than_one_gpu_is_refused(extra):
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"] + extra,
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "single GPU" in r.stderr
    assert r.stdout == ""


def test_quadrant_sizes():
    """512^2 coarse with the central 256^2 refined at r = 2: 196,608 active
    coarse cells plus 2 x 512^2 fine updates, and 1024^2 x 2 fine-equivalent
    updates per coarse step."""
    case = bench.build_case("quadrant512", 1)
    assert bench.actual_updates_per_step(case) == 196_608 + 2 * 512 * 512 == 720_896
    assert case.fine_equivalent_per_coarse_step() == 1024 * 1024 * 2


def test_uniform_sizes():
    case = bench.build_case("uniform4096", 1)
    assert bench.actual_updates_per_step(case) == 4096 * 4096
    assert case.fine_equivalent_per_coarse_step() == 4096 * 4096


def test_unknown_workload():
    with pytest.raises(SystemExit):
        bench.build_case("no-such-workload", 1)


def test_cpu_baseline_reports_its_host():
    """The oracle leg on a tiny workload: a positive rate, one thread, and the
    host CPU it ran on."""
    from paper_2609_35529_amd import workloads as wl
    r = bench.cpu_baseline(wl.sod_2d(steps=3), budget_s=5.0)
    assert r["value"] > 0 and r["cores"] == 1 and r["kind"] == "oracle"
    assert r["host"]["logical_cpus"] >= 1 and r["host"]["available_to_process"] >= 1
    assert "first 3 coarse steps" in r["sample"]
