"""Host-side hierarchy code of the 3-D path without a GPU: a check program
(tests/host/cluster3_check.cpp) built around the library's host source with
AddressSanitizer, exercising clustering, nesting, geometry and the tile and
task lists built on worker threads."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


@pytest.mark.skipif(not shutil.which(HIPCC) and not os.path.exists(HIPCC), reason="hipcc not available")
def test_clustering_and_lists_under_asan(tmp_path):
    exe = str(tmp_path / "cluster3_check")
    cmd = [HIPCC, "-std=c++17", "-O1", "-g", "-Xarch_host", "-fsanitize=address", "-fno-gpu-sanitize",
           "--cuda-host-only", "-I" + os.path.join(ROOT, "include"),
           os.path.join(HERE, "host", "cluster3_check.cpp"), "-o", exe, "-lpthread"]
    subprocess.run(cmd, check=True, capture_output=True, timeout=300)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=1")
    res = subprocess.run([exe], capture_output=True, text=True, timeout=600, env=env)
    assert res.returncode == 0, res.stdout + res.stderr
    assert res.stdout.strip().endswith("ok"), res.stdout
