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
    import mrsdc_inputs as mi
    pb = mi.machine_310k(nsteps=1)
    v = bench.counter_traffic(pb)
    c = bench.COUNTER_TRAFFIC
    # a figure only while the kernel source is the one it was measured on
    assert v is None or v == pytest.approx(
        (c["fetch_kib"] * c["fetch_scale"] + c["write_kib"] * c["write_scale"]) * 1024.0)
    other = mi.machine_310k(nsteps=1).with_scheme(precision=1 - c["precision"])
    assert bench.counter_traffic(other) is None
