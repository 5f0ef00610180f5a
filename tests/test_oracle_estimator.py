"""Pins of the oracle's estimator, sampler and grid decoding (CPU only).

Estimate (paper Sec. 2, Eq. (1), direct Monte Carlo): f = V * mean of
g(y_s; x) over n uniform samples; sigma = V * sqrt(M2 / (n (n-1))).
"""
import numpy as np
import pytest

from oracle import oracle as zo
from paper_1910_01965_amd.workloads import ScanSpec

from closed_forms import volume


def test_const_family_is_exact_volume():
    # g = 1: every sample equals 1, so f is exactly the box volume, sigma 0
    rng = np.random.default_rng(0)
    for N in (1, 2, 5, 8, 16):
        lo = rng.uniform(-3, 3, N)
        hi = lo + rng.uniform(0.1, 2.0, N)
        spec = ScanSpec("const", [np.arange(3.0), np.arange(2.0)], lo, hi, 64, 11)
        f, s = zo.scan(spec)
        assert np.all(f == np.prod(hi - lo)) and np.all(s == 0.0)


def test_two_samples_special_case():
    # n = 2: mean (v0+v1)/2, M2 = (v0-v1)^2/2, sigma = V |v0 - v1| / 2
    spec = ScanSpec("sin_sum", [np.linspace(0, 1, 7)], np.zeros(3), np.array([1.0, 2.0, 0.5]), 2, 9)
    V = volume(spec)
    f, s = zo.scan(spec)
    for g in range(spec.G):
        v0, v1 = zo.values(spec, g)
        assert f[g] == pytest.approx(V * (v0 + v1) / 2.0, rel=1e-15, abs=1e-300)
        assert s[g] == pytest.approx(V * abs(v0 - v1) / 2.0, rel=1e-13)


def test_moments_match_library_routines():
    spec = ScanSpec("gauss", [np.linspace(0.1, 10, 4), np.linspace(0.1, 10, 3)],
                    np.zeros(3), np.ones(3), 1000, 42)
    V = volume(spec)
    f, s = zo.scan(spec)
    for g in range(spec.G):
        v = zo.values(spec, g)
        mean, m2 = zo.moments(spec, g)
        assert mean == pytest.approx(float(np.mean(v)), rel=1e-14)
        assert m2 == pytest.approx(float(np.var(v) * len(v)), rel=1e-12)
        assert f[g] == pytest.approx(V * np.mean(v), rel=1e-14)
        assert s[g] == pytest.approx(V * np.std(v, ddof=1) / np.sqrt(len(v)), rel=1e-12)


def test_prefix_property_and_subset_scan():
    # values of the first k samples do not depend on n; subset = full scan rows
    spec = ScanSpec("cosexp", [np.linspace(-1, 1, 3)] * 4, np.zeros(2), np.array([2.0, 1.0]), 256, 5)
    v_all = zo.values(spec, 17)
    v_pre = zo.values(spec.with_(samples=64), 17)
    assert np.array_equal(v_all[:64], v_pre)
    assert np.array_equal(zo.values(spec, 17, 100, 20), v_all[100:120])
    f, s = zo.scan(spec)
    idx = np.array([80, 0, 17, 17, 3], dtype=np.uint64)
    fi, si = zo.scan(spec, idx)
    assert np.array_equal(fi, f[idx.astype(np.int64)]) and np.array_equal(si, s[idx.astype(np.int64)])


def test_grid_decoding_is_c_order():
    # Distinct value lists per axis, shape (2, 3, 1, 4): flat index
    # g = ((i1*3 + i2)*1 + i3)*4 + i4 (last axis fastest).  With x3 = 0 the
    # COSEXP integrand is cos(x1 y1 + x2 y2) + x4; y1 and y2 of each sample
    # are read off two LINEAR scans of the same stream in which the other
    # coordinate's edge is negligible (below half an ulp of the sum).
    axes = [np.array([-0.5, 0.5]), np.array([0.0, 0.25, -0.25]), np.array([0.0]),
            np.array([10.0, 20.0, 30.0, 40.0])]
    spec = ScanSpec("cosexp", axes, np.zeros(2), np.array([2.0, 1.0]), 8, 1)
    only_y1 = spec.with_(family="linear", hi=np.array([2.0, 1e-30]))
    only_y2 = spec.with_(family="linear", hi=np.array([1e-30, 1.0]))
    assert zo.grid_size(spec) == 24
    for g in range(spec.G):
        i1, rem = divmod(g, 12)
        i2, i4 = divmod(rem, 4)
        x1, x2, x4 = axes[0][i1], axes[1][i2], axes[3][i4]
        y1 = zo.values(only_y1, g)
        y2 = zo.values(only_y2, g)
        v = zo.values(spec, g)
        assert np.allclose(v, np.cos(x1 * y1 + x2 * y2) + x4, rtol=0, atol=1e-14)


def test_invalid_specs_rejected():
    ok = ScanSpec("gauss", [np.arange(1.0, 3.0)], np.zeros(2), np.ones(2), 16, 1)
    zo.scan(ok)
    bad = [
        ok.with_(samples=1),
        ok.with_(lo=np.array([0.0, 1.0]), hi=np.array([1.0, 1.0])),
        ok.with_(hi=np.array([1.0, np.inf])),
        ok.with_(family="cosexp"),            # needs M = 4
        ok.with_(axes=[np.arange(3.0)] * 3),  # GAUSS needs M <= N
        ok.with_(family="nope"),
        ok.with_(lo=np.zeros(17), hi=np.ones(17)),
    ]
    for b in bad:
        with pytest.raises(ValueError):
            zo.scan(b)


def test_zero_parameters_is_one_integral():
    spec = ScanSpec("sin_sum", [], np.zeros(2), np.ones(2), 128, 3)
    assert zo.grid_size(spec) == 1
    f, s = zo.scan(spec)
    assert f.shape == (1,) and np.isfinite(f[0]) and s[0] > 0
