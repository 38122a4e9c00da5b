"""CPU checks of bench.py's command line: more than one GPU is refused before
anything touches a device."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and "--gpus 2" in r.stderr
    assert r.stdout == ""


def test_traffic_figure_is_null_once_the_kernel_changes():
    sys.path.insert(0, ROOT)
    import bench
    sig = bench.kernel_signature()
    assert len(sig) == 16 and sig == bench.kernel_signature()
    saved = dict(bench.TRAFFIC_COUNTERS)
    try:
        bench.TRAFFIC_COUNTERS["x"] = (100.0, 10.0, 2.0, 1.0, sig)
        assert bench.traffic_bytes("x") == (200.0 + 10.0) * 1024
        bench.TRAFFIC_COUNTERS["x"] = (100.0, 10.0, 2.0, 1.0, "0" * 16)
        assert bench.traffic_bytes("x") is None
        assert bench.traffic_bytes("no such workload") is None
    finally:
        bench.TRAFFIC_COUNTERS.clear()
        bench.TRAFFIC_COUNTERS.update(saved)
