"""Host-side checks of the benchmark driver's contract (no GPU needed)."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.parametrize("n", [2, 8])
def test_more_than_one_gpu_is_refused(n):
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", str(n)],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU only" in r.stderr
    assert r.stdout == ""


def test_counter_traffic_only_for_its_workload():
    sys.path.insert(0, ROOT)
    import bench
    for (workload, prec), c in bench.COUNTER_TRAFFIC.items():
        v = bench.counter_traffic(workload, prec)
        # a figure only while the kernel source is the one it was measured on
        assert v is None or v == pytest.approx(
            (c["fetch_kib"] * c["fetch_scale"] + c["write_kib"] * c["write_scale"]) * 1024.0)
        assert bench.counter_traffic(workload, 1 - prec) is None or \
            (workload, 1 - prec) in bench.COUNTER_TRAFFIC
    assert bench.counter_traffic("no-such-workload", 0) is None


def test_default_headline_is_the_ensemble():
    """Without flags the bench times the 64-member 7.5 mm ensemble in the
    FP32 + refinement form (the largest single-GPU workload)."""
    sys.path.insert(0, ROOT)
    import bench
    old = sys.argv
    sys.argv = ["bench.py"]
    try:
        a = bench.parse()
    finally:
        sys.argv = old
    assert a.config == "ensemble" and a.precision is None and a.gpus == 1
