"""Host-side logic of bench.py (CPU): the one-GPU guard and the HBM traffic
read from the committed counter summaries, which is valid only for the
collide-kernel sources it was measured on."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


@pytest.mark.parametrize("workload,precision,algorithmic", [
    ("hindered384", "fp32", 2 * 19 * 4 * 384 ** 3),
    ("mixed256", "fp16s", 2 * 19 * 2 * 256 ** 3),
])
def test_committed_traffic_matches_current_kernel(workload, precision, algorithmic):
    """The counter summaries of the benchmark's workload (hindered384, FP32)
    and of the FP16-storage workload were taken on the current collide
    sources, and the measured bytes lie within 3 % above the algorithmic
    2 x 19 x s per cell (the pull halo rows are read once per XCD)."""
    t = bench.load_traffic(workload, precision)
    assert t is not None, "profile taken on other kernel sources: re-take the counters"
    assert algorithmic <= t <= 1.03 * algorithmic


def test_traffic_is_none_for_other_sources(monkeypatch):
    monkeypatch.setattr(bench, "kernel_source_hash", lambda: "0000000000000000")
    assert bench.load_traffic("spheres128", "fp32") is None
    assert bench.load_traffic("no_such_workload", "fp32") is None
