"""Host-side checks of bench.py that need no GPU: the one-GPU refusal and the counter-summary lookups."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_traffic_lookups_follow_the_measured_shape():
    import bench
    # the product's counters hold for 1024 vectors at m = 32 only
    assert bench._traffic_fft(512, 32) is None
    assert bench._traffic_fft(1024, 16) is None
    v = bench._traffic_fft(1024, 32)
    assert v is None or 1.2e9 < v < 2.0e9          # None once cg.hip differs from the measured source
    assert bench._traffic("k_unknown", 10) is None
