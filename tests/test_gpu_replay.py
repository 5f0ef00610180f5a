"""The paper's own workloads through the GPU library (needs an MI355X): the
Table 1 error column on the GPU path, and one Eq. (4) batch."""
import sys

import numpy as np
import pytest

from paper_1910_01965_amd import replay as rp

import closed_forms as cf

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1910_01965_amd import zmc
    zmc.load()
    return torch


def _spread(spec):
    """Expected dr of crude MC and its standard deviation, from the exact
    variances (dr averages |Normal| / |f_th| over the grid)."""
    f_th, var = cf.exact(spec)
    r = cf.volume(spec) * np.sqrt(var / spec.samples) / np.abs(f_th)
    return np.mean(np.sqrt(2 / np.pi) * r), np.sqrt(np.sum(r ** 2) * (1 - 2 / np.pi)) / len(r)


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_table1_error_column(precision):
    """Table 1, M = 1 and 2, N = 1..4: the GPU path's dr lies within the
    crude-MC spread of its expectation and of the printed value (the printed
    values match 10^5 samples, see the oracle's Table 1 pin)."""
    for M in (1, 2):
        for N in (1, 2, 3, 4):
            spec = rp.eq2_spec(M, N, 100_000, precision)
            f, _, t = rp.timed_scan(spec)
            dr = rp.delta_r(f, rp.sin_sum_exact(rp.grid_sum(spec), spec.lo, spec.hi))
            expect, sd = _spread(spec)
            printed = rp.PAPER_TABLE1[(M, N)][0]
            print(f"M={M} N={N} {precision}: dr {dr:.5f} expect {expect:.5f} +- {sd:.5f} "
                  f"printed {printed} ({t['eval_s'] * 1e3:.2f} ms)", flush=True)
            sys.stdout.flush()
            assert abs(dr - expect) < 4 * sd
            assert abs(dr - printed) < 4 * np.sqrt(2) * sd


def test_eq4_batch():
    """One 10^6-point batch of Eq. (4) at reduced samples: dr within the
    crude-MC spread, every value finite."""
    spec = rp.eq4_spec(4096, "fp32", x1=3)
    f, s, t = rp.timed_scan(spec)
    assert np.all(np.isfinite(f)) and np.all(np.isfinite(s)) and np.all(s > 0)
    dr = rp.delta_r(f, rp.sin_sum_exact(rp.grid_sum(spec), spec.lo, spec.hi))
    expect, sd = _spread(spec)
    print(f"eq4 batch: dr {dr:.5f} expect {expect:.5f} +- {sd:.5f}, eval {t['eval_s'] * 1e3:.2f} ms",
          flush=True)
    assert abs(dr - expect) < 4 * sd
