"""The process holds exactly one HIP runtime once the binding is loaded."""
import os


def _loaded_hip_runtimes():
    libs = set()
    with open("/proc/self/maps") as f:
        for line in f:
            path = line.split()[-1] if len(line.split()) >= 6 else ""
            if "libamdhip64" in os.path.basename(path):
                libs.add(os.path.realpath(path))
    return libs


def test_single_hip_runtime():
    from paper_2609_35529_amd import vlbm  # noqa: F401
    libs = _loaded_hip_runtimes()
    assert len(libs) == 1, libs
