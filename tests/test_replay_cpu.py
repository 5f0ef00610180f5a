"""Host parts of the paper-workload replays (no GPU): the closed form of
Eq. (2)/(4), the grid order, and the dr map of Eq. (5)."""
import numpy as np

from paper_1910_01965_amd import replay as rp
from paper_1910_01965_amd import workloads as wl

import closed_forms as cf


def test_closed_form_matches_independent_formula():
    rng = np.random.default_rng(3)
    for N in (1, 2, 4, 6):
        lo = rng.uniform(-2, 1, N)
        hi = lo + rng.uniform(0.1, 10, N)
        spec = wl.ScanSpec("sin_sum", [rng.uniform(-5, 5, 7), rng.uniform(0, 3, 5)], lo, hi, 16, 1)
        a = rp.sin_sum_exact(rp.grid_sum(spec), spec.lo, spec.hi)
        b = cf.exact(spec)[0]
        assert np.max(np.abs(a - b)) < 1e-12 * max(1.0, np.max(np.abs(b)))


def test_closed_form_special_values():
    # N = 1: int_0^h sin(c + y) dy = cos(c) - cos(c + h)
    c = np.linspace(-3, 3, 13)
    assert np.allclose(rp.sin_sum_exact(c, [0.0], [2.5]), np.cos(c) - np.cos(c + 2.5), atol=1e-14)
    # a full period in one direction integrates to zero
    assert np.allclose(rp.sin_sum_exact(c, [0.0, 0.0], [2 * np.pi, 1.0]), 0.0, atol=1e-14)


def test_grid_sum_is_c_order():
    spec = rp.eq2_spec(3, 2, 16, "fp64")
    spec = spec.with_(axes=[np.arange(3.0), 10 * np.arange(4.0), 100 * np.arange(2.0)])
    s = rp.grid_sum(spec)
    X = cf.grid_points(spec)
    assert np.array_equal(s, X.sum(axis=1))
    assert s[1] == 100.0 and s[2] == 10.0  # last axis fastest


def test_paper_shapes():
    assert rp.eq2_spec(4, 3, 10_000, "fp64").G == 100 ** 4
    b = rp.eq4_spec(100_000, "fp64", x1=7)
    assert b.G == 10 ** 6 and b.N == 6 and np.all(b.hi == 1.0) and b.axes[0][0] == 7.0
    assert rp.eq4_spec(100_000, "fp64").G == 10 ** 8
    assert len(rp.PAPER_TABLE1) == 16


def test_dr_map_eq5():
    spec = rp.eq4_spec(16, "fp64").with_(axes=[np.arange(3.0), np.arange(4.0), np.arange(5.0),
                                               np.arange(2.0)])
    f_th = rp.sin_sum_exact(rp.grid_sum(spec), spec.lo, spec.hi)
    rel = np.linspace(0.01, 0.2, spec.G)
    m = rp.dr_map(f_th * (1 + rel), spec)
    assert m.shape == (3, 4)
    # by hand: the mean over the (x3, x4) block of each (x1, x2)
    want = rel.reshape(3, 4, 10).mean(axis=2)
    assert np.allclose(m, want, rtol=1e-12)
    assert abs(rp.delta_r(f_th * (1 + rel), f_th) - rel.mean()) < 1e-12


def test_spread_matches_independent_variance():
    rng = np.random.default_rng(5)
    for N in (1, 3, 6):
        lo = rng.uniform(-1, 1, N)
        hi = lo + rng.uniform(0.2, 4, N)
        spec = wl.ScanSpec("sin_sum", [rng.uniform(-5, 5, 9)], lo, hi, 16, 1)
        _, var = cf.exact(spec)
        got = rp.sin_sum_spread(rp.grid_sum(spec), spec.lo, spec.hi)
        assert np.allclose(got, cf.volume(spec) * np.sqrt(var), rtol=1e-10, atol=1e-14)


def test_expected_map_matches_monte_carlo_spread():
    # a tiny Eq. (4) grid: the expected map against a simulated crude-MC map
    spec = rp.eq4_spec(1000, "fp64").with_(axes=[np.arange(2.0), np.arange(3.0), np.arange(20.0),
                                                 np.arange(20.0)])
    sx = rp.grid_sum(spec)
    f_th = rp.sin_sum_exact(sx, spec.lo, spec.hi)
    sd = rp.sin_sum_spread(sx, spec.lo, spec.hi) / np.sqrt(spec.samples)
    rng = np.random.default_rng(0)
    sims = np.mean([rp.dr_map(f_th + sd * rng.standard_normal(spec.G), spec) for _ in range(200)],
                   axis=0)
    assert np.allclose(sims, rp.expected_dr_map(spec), rtol=0.05)
