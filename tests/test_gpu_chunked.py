"""Out-of-core (chunked) scans into host memory (needs an MI355X): every
chunk runs the whole grid's decomposition, so the results equal an in-core
scan of the whole grid bit for bit; plus oracle parity on sampled points."""
import sys

import numpy as np
import pytest

from oracle import oracle as zo
from paper_1910_01965_amd import workloads as wl

import parity

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1910_01965_amd import zmc
    zmc.load()
    return torch


def _zmc():
    from paper_1910_01965_amd import zmc
    return zmc


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _in_core(spec):
    import torch
    f, s = _zmc().scan(spec)
    torch.cuda.synchronize()
    return f.cpu().numpy(), s.cpu().numpy()


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
@pytest.mark.parametrize("chunk", [10007, 65536, 0])
def test_chunked_equals_in_core_point_major(precision, chunk):
    spec = wl.gauss_2p(points_per_axis=300, samples=2051, precision=precision)
    _say(f"chunked {spec.name} {precision} chunk={chunk}")
    f, s = _zmc().scan_chunked(spec, chunk)
    fa, sa = _in_core(spec)
    assert np.array_equal(f, fa) and np.array_equal(s, sa)


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_chunked_equals_in_core_sample_major(precision):
    spec = wl.plain_fp64(points=1000, samples=1 << 14).with_(precision=precision)
    f, s = _zmc().scan_chunked(spec, 333)
    fa, sa = _in_core(spec)
    assert np.array_equal(f, fa) and np.array_equal(s, sa)
    f_ref, s_ref = zo.scan(spec)
    parity.check(f, s, f_ref, s_ref, spec.samples, precision, "chunked sample-major")


def test_chunked_pinned_outputs_and_oracle():
    import torch
    spec = wl.cosexp_4p(points_per_axis=20, samples=1024, precision="fp32")
    f = torch.empty(spec.G, dtype=torch.float64, pin_memory=True)
    s = torch.empty(spec.G, dtype=torch.float64, pin_memory=True)
    _zmc().scan_chunked(spec, 30000, f, s)
    fa, sa = _in_core(spec)
    assert np.array_equal(f.numpy(), fa) and np.array_equal(s.numpy(), sa)
    idx = np.sort(np.random.default_rng(4).choice(spec.G, 64, replace=False)).astype(np.uint64)
    f_ref, s_ref = zo.scan(spec, idx)
    ii = idx.astype(np.int64)
    parity.check(f.numpy()[ii], s.numpy()[ii], f_ref, s_ref, spec.samples, "fp32", "chunked pinned",
                 small_n=True, volume=2.0)


def test_chunked_user_integrand():
    src = ("template <typename T> __device__ T integrand(const T* y, const T* x, const T* p) {\n"
           "  return exp(-x[0] * (y[0] - p[0]) * (y[0] - p[0])) * cos(x[1] * y[1]);\n}\n")
    spec = wl.ScanSpec("user", [np.linspace(0.5, 4, 70), np.linspace(0, 3, 90)], np.zeros(2),
                       np.ones(2), 1025, 31, "fp64", source=src, params=np.array([0.25]))
    f, s = _zmc().scan_chunked(spec, 999)
    fa, sa = _in_core(spec)
    assert np.array_equal(f, fa) and np.array_equal(s, sa)


def test_chunked_many_chunks():
    """12 million points in 1M-point chunks: in-core equality and sampled
    oracle parity, every chunk boundary included."""
    spec = wl.ScanSpec("sin_sum", [np.linspace(0, 1, 4000), np.linspace(0, 2, 3000)], np.zeros(2),
                       np.ones(2), 64, 41, "fp32")
    C = 1 << 20
    f, s = _zmc().scan_chunked(spec, C)
    fa, sa = _in_core(spec)
    assert np.array_equal(f, fa) and np.array_equal(s, sa)
    edges = np.arange(C, spec.G, C)
    idx = np.unique(np.concatenate([edges - 1, edges, [0, spec.G - 1]])).astype(np.uint64)
    f_ref, s_ref = zo.scan(spec, idx)
    ii = idx.astype(np.int64)
    parity.check(f[ii], s[ii], f_ref, s_ref, spec.samples, "fp32", "chunk boundaries", small_n=True)


def test_chunked_rejects_device_outputs():
    import torch
    zmc = _zmc()
    spec = wl.gauss_2p(points_per_axis=20, samples=64, precision="fp32")
    f = torch.empty(spec.G, dtype=torch.float64, device="cuda")
    s = torch.empty(spec.G, dtype=torch.float64, device="cuda")
    with pytest.raises(zmc.ZmcError) as ei:
        zmc.scan_chunked(spec, 0, f, s)
    assert ei.value.status == 1


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_ranges_concatenate_to_the_whole_scan(precision):
    """Three ranges with boundaries inside point blocks, computed separately
    (as separate processes or devices would), and a resumed scan: all equal
    the whole-grid scan bit for bit."""
    zmc = _zmc()
    spec = wl.gauss_2p(points_per_axis=211, samples=1025, precision=precision)
    fa, sa = _in_core(spec)
    a, b = 10001, 30013
    parts = [zmc.scan_range(spec, lo, hi, chunk) for lo, hi, chunk in
             ((0, a, 4096), (a, b, 0), (b, spec.G, 7777))]
    f = np.concatenate([p[0] for p in parts])
    s = np.concatenate([p[1] for p in parts])
    assert np.array_equal(f, fa) and np.array_equal(s, sa)
    with pytest.raises(zmc.ZmcError):
        zmc.scan_range(spec, 5, 5)
    with pytest.raises(zmc.ZmcError):
        zmc.scan_range(spec, 0, spec.G + 1)


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_range_past_two_to_the_32(precision):
    """Global indices past 2^32 (a 5e9-point grid).  In 4096-point chunks the
    slice below 2^32 runs the fast counter path and the one above it the
    general path; 5000-point chunks put the points below 2^32 on the general
    path too.  Both splittings agree bitwise and meet the oracle bar, as do
    the grid's last points."""
    zmc = _zmc()
    a1, a2 = np.linspace(0.1, 10, 100000), np.linspace(0.1, 10, 50000)
    spec = wl.ScanSpec("gauss", [a1, a2], np.zeros(3), np.ones(3), 2049, 19, precision)
    T = 1 << 32
    _say(f"range past 2^32 {precision}")
    fa, sa = zmc.scan_range(spec, T - 4096, T + 4096, 4096)
    fb, sb = zmc.scan_range(spec, T - 4096, T + 4096, 5000)
    assert np.array_equal(fa, fb) and np.array_equal(sa, sb)
    f_ref, s_ref = zo.scan(spec, np.arange(T - 4096, T + 4096, dtype=np.uint64))
    parity.check(fa, sa, f_ref, s_ref, spec.samples, precision, "range across 2^32", small_n=True)
    fl, sl = zmc.scan_range(spec, spec.G - 1000, spec.G)
    f_ref, s_ref = zo.scan(spec, np.arange(spec.G - 1000, spec.G, dtype=np.uint64))
    parity.check(fl, sl, f_ref, s_ref, spec.samples, precision, "last points", small_n=True)


def test_boltzmann_shaped_grid_at_full_size():
    """The 1.89e8-point Boltzmann-shaped grid the benchmark streams (3 GB of f
    and sigma in host memory): 300 sampled points and both sides of every
    2^24-point chunk boundary against the oracle."""
    spec = wl.boltzmann_shape()
    _say(f"chunked {spec.name}: {spec.G} points")
    f, s = _zmc().scan_chunked(spec)
    assert np.all(np.isfinite(f)) and np.all(np.isfinite(s))
    C = 1 << 24
    edges = np.arange(C, spec.G, C)
    idx = np.concatenate([edges - 1, edges, [0, spec.G - 1],
                          np.random.default_rng(3).choice(spec.G, 300, replace=False)])
    idx = np.unique(idx).astype(np.uint64)
    f_ref, s_ref = zo.scan(spec, idx)
    ii = idx.astype(np.int64)
    _, _, msg = parity.check(f[ii], s[ii], f_ref, s_ref, spec.samples, "fp32", spec.name,
                             small_n=True, volume=1.0)
    _say(msg)


def test_grid_of_1e10_points_by_ranges():
    """A 10^10-point grid (160 GB of f and sigma) streamed in twenty ranges of
    5e8 points through the same two host arrays, as a caller without 160 GB
    of host memory would run it.  Each range: finite outputs, and its first
    and last points and four sampled ones against the oracle (most of the
    grid lies past 2^32, on the general counter path)."""
    zmc = _zmc()
    spec = wl.grid_1e10()
    step = 500_000_000
    f = np.empty(step)
    s = np.empty(step)
    rng = np.random.default_rng(12)
    idx_all, f_all, s_all = [], [], []
    for g0 in range(0, spec.G, step):
        g1 = min(spec.G, g0 + step)
        _say(f"grid 1e10: range [{g0}, {g1})")
        zmc.scan_range(spec, g0, g1, 0, f[: g1 - g0], s[: g1 - g0])
        assert np.all(np.isfinite(f[: g1 - g0])) and np.all(np.isfinite(s[: g1 - g0]))
        local = np.concatenate([[0, g1 - g0 - 1], rng.integers(0, g1 - g0, 4)])
        idx_all.append(g0 + local)
        f_all.append(f[local].copy())
        s_all.append(s[local].copy())
    idx = np.concatenate(idx_all).astype(np.uint64)
    f_ref, s_ref = zo.scan(spec, idx)
    _, _, msg = parity.check(np.concatenate(f_all), np.concatenate(s_all), f_ref, s_ref,
                             spec.samples, "fp32", spec.name, small_n=True, volume=1.0)
    _say(msg)
