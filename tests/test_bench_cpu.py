"""Host-side parts of the benchmark's contract (no GPU): more than one GPU is
refused with a message, and measured HBM traffic is reported only for the
launch shape and kernel sources its counter summary was taken with."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_traffic_only_for_the_profiled_configuration():
    t = bench.measured_traffic("ns111", "conp", "C", 262144, (2, 4))
    if t is None:
        # a summary taken with other kernel sources is not reported
        path = os.path.join(ROOT, "profiles", "pj_kernel_ns111_conp_C_2x4_traffic.txt")
        text = open(path).read()
        assert bench.kernel_sources_sha256() not in text
        pytest.skip("the counter summary predates the current kernel sources")
    assert 9.3e9 < t < 3e10   # at least the algorithmic bytes
    assert bench.measured_traffic("ns111", "conp", "C", 262144, (1, 2)) is None
    assert bench.measured_traffic("ns111", "conp", "C", 1000, (2, 4)) is None
    assert bench.measured_traffic("ns53", "conp", "C", 262144, (2, 4)) is None
