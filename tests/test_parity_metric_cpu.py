"""The parity metric itself (tests/parity.py), on hand-made numbers."""
import numpy as np
import pytest

import parity


def test_relative_bars():
    # err_f scales by max(|f_ref|, sigma_ref sqrt(n)); err_sigma is relative
    ef, es = parity.errors([1.0 + 1e-13], [0.01 * (1 + 1e-13)], [1.0], [0.01], 100)
    assert ef[0] == pytest.approx(1e-13, rel=1e-2) and es[0] == pytest.approx(1e-13, rel=1e-2)
    # f_ref = 0: judged against the integrand's own scale sigma_ref sqrt(n)
    ef, _ = parity.errors([1e-3], [0.1], [0.0], [0.1], 10000)
    assert ef[0] == pytest.approx(1e-4)


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_constant_integrand_needs_sigma_within_1e_12_of_f(precision):
    # sigma_ref = 0: sigma <= 1e-12 |f_ref| in both precisions
    parity.check([2.0], [0.0], [2.0], [0.0], 16, precision)
    parity.check([2.0], [1.9e-12], [2.0], [0.0], 16, precision)
    with pytest.raises(AssertionError):
        parity.check([2.0], [2.1e-12], [2.0], [0.0], 16, precision)
    # f_ref = sigma_ref = 0 leaves no room at all
    with pytest.raises(AssertionError):
        parity.check([0.0], [1e-300], [0.0], [0.0], 16, precision)


def test_small_n_floor_is_fp32_only_and_below_4096_samples():
    n, V = 16, 1.0
    floor_abs = 2.0 ** -18 * V * (1.0 + 1.0) / np.sqrt(n)  # allowance at f_ref = V
    s_ref = 1e-9                                            # a nearly constant sample set
    s = s_ref + 0.9 * floor_abs
    parity.check([1.0], [s], [1.0], [s_ref], n, "fp32", small_n=True)
    with pytest.raises(AssertionError):  # the plain relative bar
        parity.check([1.0], [s], [1.0], [s_ref], n, "fp32")
    with pytest.raises(AssertionError):  # beyond the allowance
        parity.check([1.0], [s_ref + 1.1 * floor_abs], [1.0], [s_ref], n, "fp32", small_n=True)
    with pytest.raises(AssertionError):  # the FP64 path never takes the floor
        parity.check([1.0], [s], [1.0], [s_ref], n, "fp64", small_n=True)
    with pytest.raises(ValueError):
        parity.errors([1.0], [s], [1.0], [s_ref], 4096, "fp32", small_n=True)
