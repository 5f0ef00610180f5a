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


def test_serving_window_fits_the_time_budget():
    # 200 req/s of ~8.6e9-sample requests: about 1.7e12 samples per second of arrivals
    sys.path.insert(0, ROOT)
    import bench

    def trace(sec):
        return 1.72e12 * sec

    # 60 s of arrivals: 1.03e14 samples, ~145 s served and ~145 s replayed at 7.1e11/s
    assert bench.fit_serving_window(60.0, 470.0, 7.1e11, 7.1e11, 4.0, trace) == 60.0
    # less time left: the window halves until the section fits, never below 4 s
    assert bench.fit_serving_window(60.0, 250.0, 7.1e11, 7.1e11, 4.0, trace) == 30.0
    assert bench.fit_serving_window(60.0, 10.0, 7.1e11, 7.1e11, 4.0, trace) == 4.0


def test_mix_roofline_weights_each_scan_by_its_samples():
    sys.path.insert(0, ROOT)
    import bench
    from paper_1910_01965_amd import workloads as wl
    a = wl.gauss_2p(points_per_axis=10, samples=1024)            # 51 ops per sample
    b = wl.cosexp_4p(precision="fp32").with_(samples=4096)
    b = b.with_(axes=[ax[:3] for ax in b.axes])                  # 81 points, 39 ops per sample
    r = bench.mix_roofline([a, b], 2.0)
    ops = 100 * 1024 * 51 + 81 * 4096 * 39
    assert r["bound"] == "alu"
    assert abs(r["frac"] - ops / 2.0 / bench.VALU_PEAK) < 1e-15
    assert abs(r["ops_per_sample_mean"] - ops / (100 * 1024 + 81 * 4096)) < 1e-12


def test_serving_window_counts_a_long_shortest_first_run():
    sys.path.insert(0, ROOT)
    import bench

    def trace(sec):
        return 1.72e12 * sec

    # a 60 s shortest-first run costs another ~145 s: 60 s no longer fits 470 s
    assert bench.fit_serving_window(60.0, 470.0, 7.1e11, 7.1e11, 60.0, trace) == 30.0
    assert bench.fit_serving_window(60.0, 900.0, 7.1e11, 7.1e11, 60.0, trace) == 60.0
