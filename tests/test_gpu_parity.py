"""GPU library vs the oracle, through the C ABI (needs an MI355X).

FP64 path: |f - f_ref| and |sigma - sigma_ref| within 1e-12 of their scales
(tests/parity.py); FP32-evaluation path: 2e-5 on f, 1e-3 on sigma.  Sizes
range from tiny ragged cases to the full 1e6- and 1e8-point grids, where the
oracle checks sampled points one by one.
"""
import sys

import numpy as np
import pytest

from oracle import oracle as zo
from paper_1910_01965_amd import workloads as wl

import closed_forms as cf
import parity

pytestmark = pytest.mark.gpu


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


def _run(spec, **kw):
    import torch
    f, s = _zmc().scan(spec, **kw)
    torch.cuda.synchronize()
    return f.cpu().numpy(), s.cpu().numpy()


# ---------------------------------------------------------------- words ----
@pytest.mark.parametrize("seed,g,w0,count", [
    (42, 0, 0, 4096),
    (42, 999, 1, 1000),
    (0xDEADBEEFCAFEF00D, (1 << 33) + 17, 12, 333),
    (1, 3, (1 << 34) + 8, 64),
    (0xFFFFFFFFFFFFFFFF, (1 << 64) - 1, 4 * ((1 << 32) - 1), 64),
])
def test_device_words_match_oracle(seed, g, w0, count):
    _say(f"words seed={seed} g={g} w0={w0} count={count}")
    got = _zmc().debug_words(seed, g, w0, count).cpu().numpy()
    ref = np.array([zo.word(seed, g, w0 + i) for i in range(count)], dtype=np.int64)
    assert np.array_equal(got, ref)


# --------------------------------------------------------------- values ----
def _family_specs(precision):
    out = []
    for N in range(1, 9):
        out.append(wl.ScanSpec("sin_sum", [np.linspace(0, 1, 5)], np.zeros(N), np.linspace(1, 2, N),
                               64, 7, precision))
        M = min(2, N)
        out.append(wl.ScanSpec("gauss", [np.linspace(0.1, 10, 3)] * M, -0.5 * np.ones(N),
                               np.linspace(1, 2, N), 64, 8, precision))
        if N >= 2:
            hi = np.ones(N)
            hi[0] = 2.0
            out.append(wl.ScanSpec("cosexp", [np.linspace(-1, 1, 3)] * 4, np.zeros(N), hi, 64, 9,
                                   precision))
        out.append(wl.ScanSpec("linear", [np.arange(3.0)], -np.ones(N), np.linspace(0.5, 3, N), 64,
                               10, precision))
        out.append(wl.ScanSpec("const", [np.arange(2.0)], np.zeros(N), np.ones(N), 64, 11, precision))
    return out


@pytest.mark.parametrize("spec", _family_specs("fp64"), ids=lambda s: f"{s.family}-N{s.N}")
def test_device_values_fp64_match_oracle(spec):
    _say(f"values fp64 {spec.family} N={spec.N}")
    for g in (0, spec.G - 1):
        got = _zmc().debug_values(spec, g, 3, 61).cpu().numpy()
        ref = zo.values(spec, g, 3, 61)
        assert np.allclose(got, ref, rtol=1e-14, atol=1e-15), (g, np.max(np.abs(got - ref)))


@pytest.mark.parametrize("spec", _family_specs("fp32"), ids=lambda s: f"{s.family}-N{s.N}")
def test_device_values_fp32_close_to_oracle(spec):
    _say(f"values fp32 {spec.family} N={spec.N}")
    for g in (0, spec.G - 1):
        got = _zmc().debug_values(spec, g, 0, 64).cpu().numpy()
        ref = zo.values(spec, g, 0, 64)
        scale = 1.0 + np.abs(ref)
        assert np.all(np.abs(got - ref) <= 4e-6 * scale * spec.N), (g, np.max(np.abs(got - ref)))


# ------------------------------------------------------- whole scans -------
def test_plain_fp64_full_grid():
    spec = wl.plain_fp64()
    _say(f"scan {spec.name}")
    f, s = _run(spec)
    f_ref, s_ref = zo.scan(spec)
    _, _, msg = parity.check(f, s, f_ref, s_ref, spec.samples, "fp64", spec.name)
    _say(msg)


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_gauss_reduced_grid(precision):
    spec = wl.gauss_2p(points_per_axis=40, samples=1 << 14, precision=precision)
    _say(f"scan {spec.name} {precision}")
    f, s = _run(spec)
    f_ref, s_ref = zo.scan(spec)
    _, _, msg = parity.check(f, s, f_ref, s_ref, spec.samples, precision, spec.name)
    _say(msg)


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_cosexp_reduced_grid(precision):
    spec = wl.cosexp_4p(points_per_axis=7, samples=4096, precision=precision)
    _say(f"scan {spec.name} {precision}")
    f, s = _run(spec)
    f_ref, s_ref = zo.scan(spec)
    _, _, msg = parity.check(f, s, f_ref, s_ref, spec.samples, precision, spec.name)
    _say(msg)


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_gauss_full_grid_sampled(precision):
    spec = wl.gauss_2p(precision=precision)
    _say(f"scan {spec.name} full grid {precision}")
    f, s = _run(spec)
    idx = np.sort(np.random.default_rng(1).choice(spec.G, 300, replace=False))
    idx = np.concatenate([[0, spec.G - 1], idx]).astype(np.uint64)
    f_ref, s_ref = zo.scan(spec, idx)
    ii = idx.astype(np.int64)
    _, _, msg = parity.check(f[ii], s[ii], f_ref, s_ref, spec.samples, precision, spec.name)
    _say(msg)
    # at any size: every point against the exact integral and standard error
    f_true, var = cf.gauss_exact(spec)
    ok, cmsg = cf.coverage_ok((f - f_true) / np.sqrt(var / spec.samples), spec.name)
    ratio = s / np.sqrt(var / spec.samples)
    assert abs(np.median(ratio) - 1.0) < 0.01, np.median(ratio)
    _say(cmsg)
    assert ok, cmsg


def test_gauss_full_grid_every_point():
    """The 1e6-point Gaussian grid at 2^14 samples, every point of both GPU
    paths against the oracle.  The oracle runs on up to 16 host threads
    (its C calls release the interpreter lock; it keeps no shared state)."""
    import concurrent.futures as cfut
    import os
    spec = wl.gauss_2p(precision="fp64")
    f64, s64 = _run(spec)
    f32, s32 = _run(spec.with_(precision="fp32"))
    parts = np.array_split(np.arange(spec.G, dtype=np.uint64), 128)
    workers = max(1, min(16, os.cpu_count() or 1))
    _say(f"oracle on all {spec.G} points, {workers} threads")
    with cfut.ThreadPoolExecutor(workers) as ex:
        res = list(ex.map(lambda idx: zo.scan(spec, idx), parts))
    f_ref = np.concatenate([r[0] for r in res])
    s_ref = np.concatenate([r[1] for r in res])
    for f, s, prec in ((f64, s64, "fp64"), (f32, s32, "fp32")):
        _, _, msg = parity.check(f, s, f_ref, s_ref, spec.samples, prec, f"{spec.name} every point")
        _say(msg)


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_cosexp_full_grid_subsample(precision):
    spec = wl.cosexp_4p(precision=precision)
    _say(f"scan {spec.name} full grid {precision}")
    import torch
    f, s = _zmc().scan(spec)
    idx = wl.cosexp_subsample()
    ti = torch.from_numpy(idx.astype(np.int64)).cuda()
    fs, ss = f[ti].cpu().numpy(), s[ti].cpu().numpy()
    assert bool(torch.isfinite(f).all()) and bool(torch.isfinite(s).all())
    del f, s
    f_ref, s_ref = zo.scan(spec, idx)
    _, _, msg = parity.check(fs, ss, f_ref, s_ref, spec.samples, precision, spec.name + " subsample")
    _say(msg)


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("mode", ["point_major", "sample_major"])
def test_eq2_large_phases(precision, mode):
    """The paper's Eq. (2) integrand at its Table 1 extent (M = N = 4, x_l in
    0..99, y in [0,10]^4): phases up to 436 rad, about 69 revolutions, so the
    FP64 sine's reduction and fold run far from the origin on both branches."""
    axis = np.array([0.0, 17.0, 38.0, 59.0, 80.0, 99.0])
    spec = wl.ScanSpec("sin_sum", [axis] * 4, np.zeros(4), np.full(4, 10.0), 4099, 21, precision)
    _say(f"eq2 large phases {precision} {mode} G={spec.G}")
    f, s = _run(spec, mode=mode)
    f_ref, s_ref = zo.scan(spec)
    _, _, msg = parity.check(f, s, f_ref, s_ref, spec.samples, precision, f"eq2 {mode}")
    _say(msg)


# --------------------------------------------- decomposition, edge cases ----
DECOMPOSITIONS = [
    dict(mode="point_major", splits=1), dict(mode="point_major", splits=3),
    dict(mode="point_major", block=64, splits=7), dict(mode="sample_major", splits=1),
    dict(mode="sample_major", block=64, splits=2), dict(mode="sample_major", block=1024, splits=5),
    dict(),
]


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_decomposition_invariance(precision):
    spec = wl.gauss_2p(points_per_axis=19, samples=4099, precision=precision)
    f_ref, s_ref = zo.scan(spec)
    outs = []
    for kw in DECOMPOSITIONS:
        _say(f"decomposition {kw} {precision}")
        f, s = _run(spec, **kw)
        parity.check(f, s, f_ref, s_ref, spec.samples, precision, f"{kw}")
        outs.append((f, s))
    tol = 1e-13 if precision == "fp64" else 2e-6
    for f, s in outs[1:]:
        assert np.allclose(f, outs[0][0], rtol=tol, atol=tol * np.abs(outs[0][0]).max())


def test_repeatable_bitwise():
    for precision in ("fp64", "fp32"):
        spec = wl.gauss_2p(points_per_axis=300, samples=1024, precision=precision)
        _say(f"repeat {spec.name}")
        a = _run(spec)
        b = _run(spec)
        assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("mode", ["point_major", "sample_major"])
def test_gauss_signed_coefficients(precision, mode):
    """GAUSS with negative, zero and positive coefficients on one grid: waves
    of all-nonnegative points take the reduced form, mixed waves the general
    one; both against the oracle."""
    # 60 points per row: waves straddle rows, so rows with x1 < 0 next to rows
    # with x1 >= 0 give mixed waves; x2 starts at exactly 0
    spec = wl.ScanSpec("gauss", [np.linspace(-0.6, 2.0, 41), np.linspace(0.0, 1.5, 60)],
                       np.array([-0.5, 0.0, -1.0]), np.array([1.0, 1.5, 0.5]), 2048, 12, precision)
    _say(f"gauss signed coefficients {precision} {mode}")
    f, s = _run(spec, mode=mode)
    f_ref, s_ref = zo.scan(spec)
    _, _, msg = parity.check(f, s, f_ref, s_ref, spec.samples, precision, spec.name)
    _say(msg)
    for g in (0, 30 * 60, spec.G - 1):  # x1 < 0; x1 > 0 with x2 = 0; both > 0
        got = _zmc().debug_values(spec, g, 5, 40).cpu().numpy()
        ref = zo.values(spec, g, 5, 40)
        tol = 1e-14 if precision == "fp64" else 4e-6 * spec.N
        assert np.all(np.abs(got - ref) <= tol * (1.0 + np.abs(ref))), g


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_gauss_point_independent_of_its_wave(precision):
    """A point's result does not depend on the other points of its wave:
    making one coefficient of a 256-point grid negative moves that wave off
    the reduced form, and every other point keeps its bits."""
    xs = np.linspace(0.05, 4.0, 256)
    a = wl.ScanSpec("gauss", [xs], np.zeros(3), np.ones(3), 4096, 13, precision)
    ys = xs.copy()
    ys[70] = -0.5
    b = a.with_(axes=[ys])
    fa, sa = _run(a, mode="point_major", splits=2)
    fb, sb = _run(b, mode="point_major", splits=2)
    keep = np.arange(256) != 70
    assert np.array_equal(fa[keep], fb[keep]) and np.array_equal(sa[keep], sb[keep])
    f_ref, s_ref = zo.scan(b)
    parity.check(fb, sb, f_ref, s_ref, b.samples, precision, "gauss one negative coefficient")


EDGE = [
    wl.ScanSpec("sin_sum", [], np.zeros(3), np.ones(3), 1001, 5),            # M = 0, G = 1
    wl.ScanSpec("sin_sum", [np.linspace(0, 1, 7)], np.zeros(1), np.ones(1), 2, 5),
    wl.ScanSpec("sin_sum", [np.linspace(0, 1, 7)], np.zeros(2), np.ones(2), 3, 5),
    wl.ScanSpec("gauss", [np.linspace(0.1, 9, 300)], np.zeros(8), np.ones(8), 5, 6),
    wl.ScanSpec("cosexp", [np.linspace(-1, 1, 3)] * 4, np.zeros(5), np.array([2.0, 1, 1, 1, 1]), 1001, 7),
    wl.ScanSpec("linear", [np.arange(257.0)], -np.ones(7), np.ones(7), 4097, 8),
    wl.ScanSpec("gauss", [np.linspace(0.1, 9, 70000)], np.zeros(2), np.ones(2), 33, 9),
    # the largest shapes: 16 parameter axes (G = 2^16), and M = N = 8
    wl.ScanSpec("sin_sum", [np.array([0.0, 0.5 + k / 16.0]) for k in range(16)], np.zeros(8),
                np.ones(8), 33, 10),
    wl.ScanSpec("gauss", [np.linspace(0.1, 9, 3)] * 8, np.zeros(8), np.ones(8), 257, 11),
    # the descriptor's limits together: M = 16 axes and N = 16 dimensions
    wl.ScanSpec("sin_sum", [np.array([0.0, 0.25 + k / 32.0]) for k in range(16)], -np.ones(16),
                np.linspace(0.5, 1.0, 16), 33, 12),
    wl.ScanSpec("gauss", [np.array([0.2, 1.0 + k / 8.0]) for k in range(16)], np.zeros(16),
                np.ones(16), 17, 13),
]


@pytest.mark.parametrize("spec", EDGE, ids=lambda s: f"{s.family}-G{s.G}-N{s.N}-n{s.samples}")
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("mode", ["auto", "point_major", "sample_major"])
def test_edge_shapes(spec, precision, mode):
    spec = spec.with_(precision=precision)
    _say(f"edge {spec.family} G={spec.G} N={spec.N} n={spec.samples} {precision} {mode}")
    f, s = _run(spec, mode=mode)
    f_ref, s_ref = zo.scan(spec)
    parity.check(f, s, f_ref, s_ref, spec.samples, precision, f"edge {mode}",
                 small_n=spec.samples < 4096, volume=float(np.prod(spec.hi - spec.lo)))


def test_const_is_exact_volume_on_gpu():
    for precision in ("fp64", "fp32"):
        spec = wl.ScanSpec("const", [np.arange(5.0)], np.array([-1.0, 0.5]), np.array([2.0, 1.75]),
                           999, 1, precision)
        f, s = _run(spec)
        assert np.all(f == 3.0 * 1.25) and np.all(s == 0.0)


def test_host_entry_point_matches_device():
    spec = wl.gauss_2p(points_per_axis=33, samples=2048, precision="fp32")
    _say("host entry point")
    fd, sd = _run(spec)
    fh, sh = _zmc().scan_host(spec)
    assert np.array_equal(fd, fh) and np.array_equal(sd, sh)


def test_in_core_scan_past_two_to_the_32():
    """An in-core scan of 2^32 + 2^16 points (69 GB of outputs): local and
    global indices past 2^32 on the general counter path.  Sampled points at
    the start, around 2^32 and at the end meet the oracle bar."""
    import torch
    zmc = _zmc()
    a1, a2 = np.linspace(0.1, 10, (1 << 16) + 1), np.linspace(0.1, 10, 1 << 16)
    spec = wl.ScanSpec("gauss", [a1, a2], np.zeros(3), np.ones(3), 5, 23, "fp32")
    T = 1 << 32
    assert spec.G == T + (1 << 16)
    assert zmc.plan(spec)["mode"] == "point_major"
    _say(f"in-core scan of {spec.G} points")
    f, s = zmc.scan(spec)
    torch.cuda.synchronize()
    idx = np.concatenate([np.arange(0, 100), np.arange(T - 100, T + 100), np.arange(spec.G - 100, spec.G)])
    ii = torch.from_numpy(idx).cuda()
    fg, sg = f[ii].cpu().numpy(), s[ii].cpu().numpy()
    del f, s
    torch.cuda.empty_cache()
    f_ref, s_ref = zo.scan(spec, idx.astype(np.uint64))
    parity.check(fg, sg, f_ref, s_ref, spec.samples, "fp32", "in-core past 2^32", small_n=True, volume=1.0)


def test_integrate_front_end():
    """zmc.integrate (integrand, domain, parameter lists) gives the results of
    the descriptor entry points, shaped like the grid, on the host and on the
    device; a source integrand with constants meets the oracle bar."""
    zmc = _zmc()
    ax = np.linspace(0.1, 10.0, 60)
    spec = wl.gauss_2p(points_per_axis=60, samples=2048, precision="fp32")
    f, s = zmc.integrate("gauss", [(0.0, 1.0)] * 3, [ax, ax], 2048, seed=42, precision="fp32")
    assert f.shape == (60, 60) and s.shape == (60, 60) and isinstance(f, np.ndarray)
    fa, sa = _run(spec)
    assert np.array_equal(f.ravel(), fa) and np.array_equal(s.ravel(), sa)
    fd, sd = zmc.integrate("gauss", [(0.0, 1.0)] * 3, [ax, ax], 2048, seed=42, precision="fp32",
                           host=False)
    assert fd.is_cuda and tuple(fd.shape) == (60, 60)
    assert np.array_equal(fd.cpu().numpy(), f) and np.array_equal(sd.cpu().numpy(), s)
    src = ("template <typename T> __device__ T integrand(const T* y, const T* x, const T* p) {\n"
           "  return exp(-p[0] * x[0] * y[0] * y[0]) * cos(x[1] * y[1]);\n}\n")
    a1, a2 = np.linspace(0.5, 3.0, 7), np.linspace(0.0, 2.0, 5)
    f, s = zmc.integrate(src, [(-1.0, 1.0), (0.0, 2.0)], [a1, a2], 4099, seed=9, constants=[0.5])
    ref = wl.ScanSpec("user", [a1, a2], np.array([-1.0, 0.0]), np.array([1.0, 2.0]), 4099, 9,
                      "fp64", source=src, params=np.array([0.5]))
    f_ref, s_ref = zo.scan(ref)
    parity.check(f.ravel(), s.ravel(), f_ref, s_ref, ref.samples, "fp64", "integrate, source")
    f0, s0 = zmc.integrate("sin_sum", [(0.0, 1.0)] * 2, [], 1000, seed=3)   # M = 0: one integral
    assert f0.shape == () and np.isfinite(f0) and s0 > 0


def test_valu_probe_runs():
    import torch
    out = _zmc().debug_valu_probe(64, 100)
    torch.cuda.synchronize()
    v = out.cpu().numpy()
    assert v.shape == (64 * 256,) and np.all(np.isfinite(v)) and np.all(v > 0)
