"""Integration dimensions N = 9..16 (needs an MI355X): these scans run in
kernels of their own (per (family, precision, N) variant), outside the
any-family batch kernel, in every entry point.

Per-sample values against the oracle's, whole scans element by element in
both layouts and both precisions, a batch mixing them with N <= 8 scans
(per-variant and one-kernel batches), and the server: each result equals its
alone result bit for bit and the oracle's to the usual bars (FP64 1e-12;
FP32 2e-5 on f, 1e-3 on sigma; sample counts >= 4096 so that no small-n
floor applies).
"""
import sys

import numpy as np
import pytest

from oracle import oracle as zo
from paper_1910_01965_amd import workloads as wl

import parity

pytestmark = pytest.mark.gpu

WIDE = (12, 16)


@pytest.fixture(scope="module", autouse=True)
def gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1910_01965_amd import zmc
    zmc.load()  # raises when the HIP library is missing: no fallback
    return torch


def _zmc():
    from paper_1910_01965_amd import zmc
    return zmc


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _spec(family, N, precision, points=5, samples=4099, seed=0):
    """A small grid of `family` at dimension N: ragged sample count, a box
    that is not the unit cube."""
    if family == "sin_sum":
        axes, lo, hi = [np.linspace(0.0, 3.0, points * 26)], -0.5 * np.ones(N), np.linspace(0.5, 1.5, N)
    elif family == "gauss":
        axes = [np.linspace(0.1, 10.0, points * 2), np.linspace(0.5, 4.0, 13)]
        lo, hi = np.zeros(N), np.linspace(0.7, 1.3, N)
    elif family == "cosexp":
        axes = [np.linspace(-1.0, 1.0, points)] * 3 + [np.array([-0.3, 0.4])]
        lo, hi = np.zeros(N), np.ones(N)
        hi[0] = 2.0
    else:
        raise ValueError(family)
    return wl.ScanSpec(family, axes, lo, hi, samples, 300 + N + 7 * seed, precision,
                       name=f"{family}_N{N}_{precision}")


def _volume(sp):
    return float(np.prod(sp.hi - sp.lo))


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("family", ["sin_sum", "gauss", "cosexp"])
@pytest.mark.parametrize("N", WIDE)
def test_wide_values_match_oracle(N, family, precision):
    sp = _spec(family, N, precision)
    _say(f"wide values {family} N={N} {precision}")
    for g in (0, sp.G - 1):
        got = _zmc().debug_values(sp, g, 5, 64).cpu().numpy()
        ref = zo.values(sp, g, 5, 64)
        if precision == "fp64":
            assert np.allclose(got, ref, rtol=1e-14, atol=1e-15), (g, np.max(np.abs(got - ref)))
        else:
            assert np.all(np.abs(got - ref) <= 4e-6 * (1.0 + np.abs(ref)) * N), (g, np.max(np.abs(got - ref)))


_REF = {}


def _oracle(sp):
    key = (sp.family, sp.N, sp.seed, sp.samples)
    if key not in _REF:
        _REF[key] = zo.scan(sp.with_(precision="fp64"))
    return _REF[key]


@pytest.mark.parametrize("mode", ["point_major", "sample_major"])
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("family", ["sin_sum", "gauss", "cosexp"])
@pytest.mark.parametrize("N", WIDE)
def test_wide_scan_matches_oracle(N, family, precision, mode):
    import torch
    sp = _spec(family, N, precision)
    pl = _zmc().plan(sp, mode=mode)
    _say(f"wide scan {family} N={N} {precision} {mode} G={sp.G} plan {pl}")
    f, s = _zmc().scan(sp, mode=mode)
    torch.cuda.synchronize()
    f_ref, s_ref = _oracle(sp)
    _, _, msg = parity.check(f.cpu().numpy(), s.cpu().numpy(), f_ref, s_ref, sp.samples, precision,
                             f"N={N} {family} {precision} {mode}", volume=_volume(sp))
    _say(msg)


def _mix():
    """Wide scans of the three families in both precisions beside N <= 8 ones."""
    out = []
    for i, (fam, N, prec) in enumerate([("gauss", 12, "fp32"), ("sin_sum", 16, "fp64"),
                                        ("cosexp", 16, "fp32"), ("cosexp", 12, "fp64"),
                                        ("sin_sum", 12, "fp32"), ("gauss", 16, "fp64"),
                                        ("gauss", 3, "fp32"), ("sin_sum", 5, "fp64")]):
        out.append(_spec(fam, N, prec, samples=4096 + 5 * i, seed=i))
    out.append(_spec("sin_sum", 16, "fp32", points=400, samples=4097, seed=9))  # point-major tiles
    return out


def _alone(sp):
    f, s = _zmc().scan_batch([sp])[0]
    return f.cpu().numpy(), s.cpu().numpy()


def _check(specs, outs, label):
    for sp, (f, s) in zip(specs, outs):
        idx = np.sort(np.random.default_rng(sp.seed).choice(sp.G, min(sp.G, 48), replace=False))
        f_ref, s_ref = zo.scan(sp.with_(precision="fp64"), idx.astype(np.uint64))
        _, _, msg = parity.check(f[idx], s[idx], f_ref, s_ref, sp.samples, sp.precision,
                                 f"{label} {sp.name} G={sp.G}", volume=_volume(sp))
        _say(msg)


@pytest.mark.parametrize("one_kernel", [False, True])
def test_wide_batch_equals_alone_and_oracle(one_kernel):
    zmc = _zmc()
    specs = _mix()
    info = zmc.batch_plan(specs, one_kernel=one_kernel)
    _say(f"wide batch one_kernel={one_kernel}: {info}")
    outs = [(f.cpu().numpy(), s.cpu().numpy()) for f, s in zmc.scan_batch(specs, one_kernel=one_kernel)]
    for sp, (f, s) in zip(specs, outs):
        fa, sa = _alone(sp)
        assert np.array_equal(f, fa) and np.array_equal(s, sa), sp.name
    _check(specs, outs, f"batch one_kernel={one_kernel}")


def test_wide_requests_in_the_server():
    import torch
    zmc = _zmc()
    specs = _mix()
    srv = zmc.Server(max_slots=4, slice_samples=1 << 24)
    tickets = [srv.submit(sp) for sp in specs]
    for t in tickets:
        st, _ = srv.wait(t)
        assert st == 0
    stats = srv.stats()
    _say(f"wide serving: {stats}")
    assert stats["completed"] == len(specs) and stats["slices"] > 1
    torch.cuda.synchronize()
    outs = []
    for sp, t in zip(specs, tickets):
        f, s = srv.outputs(t)
        f, s = f.cpu().numpy(), s.cpu().numpy()
        fa, sa = _alone(sp)
        assert np.array_equal(f, fa) and np.array_equal(s, sa), sp.name
        outs.append((f, s))
    srv.close()
    _check(specs, outs, "server")

