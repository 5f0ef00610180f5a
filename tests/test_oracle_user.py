"""The oracle's user-integrand path (family "user"), pinned to the oracle's
compiled-in families, which are pinned to closed forms elsewhere, and to
exact results: constants, the parameter vector, and the grid decoding."""
import numpy as np
import pytest

from oracle import oracle as zo
from paper_1910_01965_amd.workloads import ScanSpec

HEAD = "template <typename T> __device__ T integrand(const T* y, const T* x, const T* p) {\n"

LINEAR = HEAD + "  T s = 0;\n  for (int k = 0; k < 4; ++k) s += y[k];\n  return s;\n}\n"
GAUSS = HEAD + ("  T q = 0;\n  for (int k = 0; k < 3; ++k) { T c = k < 2 ? x[k] : T(1); q += c * y[k] * y[k]; }\n"
                "  return exp(-q);\n}\n")
CONST = HEAD + "  return T(1);\n}\n"
PARAMS = HEAD + "  return p[0] + p[1] * y[0] + p[5];\n}\n"
SECOND_X = HEAD + "  return x[1];\n}\n"


def test_user_linear_equals_compiled_family():
    a = ScanSpec("linear", [np.arange(5.0)], -np.ones(4), np.linspace(0.5, 3, 4), 1001, 8)
    u = a.with_(family="user", source=LINEAR)
    for g in (0, 4):
        assert np.array_equal(zo.values(a, g, 7, 50), zo.values(u, g, 7, 50))
    fa, sa = zo.scan(a)
    fu, su = zo.scan(u)
    assert np.array_equal(fa, fu) and np.array_equal(sa, su)


def test_user_gauss_matches_compiled_family():
    a = ScanSpec("gauss", [np.linspace(0.1, 10, 4), np.linspace(0.3, 2, 3)], np.zeros(3),
                 np.ones(3), 777, 9)
    u = a.with_(family="user", source=GAUSS)
    fa, sa = zo.scan(a)
    fu, su = zo.scan(u)
    assert np.allclose(fu, fa, rtol=1e-14, atol=0) and np.allclose(su, sa, rtol=1e-12, atol=0)


def test_user_constant_gives_volume():
    u = ScanSpec("user", [np.arange(3.0)], np.array([0.0, -1.0]), np.array([2.0, 0.5]), 64, 1,
                 source=CONST)
    f, s = zo.scan(u)
    assert np.all(f == 3.0) and np.all(s == 0.0)


def test_user_params_and_zero_fill():
    # p[0] + p[1] y over [lo, hi]: V (p0 + p1 (lo + hi) / 2) plus MC noise in
    # the p1 term only; p[5] is beyond n_params and reads 0
    u = ScanSpec("user", [], np.array([1.0]), np.array([3.0]), 4096, 2, source=PARAMS,
                 params=np.array([0.25, 0.0]))
    f, s = zo.scan(u)
    assert f[0] == 2.0 * 0.25 and s[0] == 0.0
    u = u.with_(params=np.array([0.25, 1.5]))
    f, s = zo.scan(u)
    exact = 2.0 * (0.25 + 1.5 * 2.0)
    assert abs(f[0] - exact) < 5 * s[0] and 0 < s[0] < 0.05


def test_user_sees_grid_point_in_c_order():
    u = ScanSpec("user", [np.array([1.0, 2.0]), np.array([10.0, 20.0, 30.0])], np.zeros(1),
                 np.ones(1), 16, 3, source=SECOND_X)
    f, s = zo.scan(u)
    assert np.array_equal(f, np.array([10.0, 20.0, 30.0, 10.0, 20.0, 30.0])) and np.all(s == 0.0)


def test_user_source_that_does_not_compile():
    u = ScanSpec("user", [], np.zeros(1), np.ones(1), 16, 3, source=HEAD + "  return nope;\n}\n")
    with pytest.raises(ValueError):
        zo.scan(u)
