"""Host-side behaviour of bench.py (no GPU needed)."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], cwd=ROOT,
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2 and r.stdout == ""
    assert "one GPU only" in r.stderr


def test_ops_per_sample_of_the_benchmark_integrand():
    # GAUSS at N = 3: Philox 10N, uniform map 2N, integrand 2N + 1, compensated sums 8
    sys.path.insert(0, ROOT)
    import bench
    assert bench.valu_ops_per_sample("gauss", 3) == 30 + 6 + 7 + 8
    assert bench.valu_ops_per_sample("cosexp", 2) == 20 + 4 + 7 + 8
