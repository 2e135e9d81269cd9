"""The worker pool the host code of both libraries shares
(paper_2609_35529_amd/csrc/host_util.hpp), without a GPU: a check program
(tests/host/pool_check.cpp) built with ThreadSanitizer runs flat sections of
every size up to 64, three nested levels of sections and sections started by
four host threads at once, and checks that every item ran exactly once."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
CXX = shutil.which("g++")


@pytest.mark.skipif(CXX is None, reason="g++ not available")
def test_pool_sections_under_tsan(tmp_path):
    exe = str(tmp_path / "pool_check")
    cmd = [CXX, "-std=c++17", "-O1", "-g", "-fsanitize=thread", os.path.join(HERE, "host", "pool_check.cpp"),
           "-o", exe, "-lpthread"]
    subprocess.run(cmd, check=True, capture_output=True, timeout=300)
    env = dict(os.environ, TSAN_OPTIONS="halt_on_error=1")
    res = subprocess.run([exe], capture_output=True, text=True, timeout=300, env=env)
    assert res.returncode == 0, res.stdout + res.stderr
    assert res.stdout.strip().endswith("ok"), res.stdout
