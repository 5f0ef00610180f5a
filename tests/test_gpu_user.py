"""User integrands compiled at run time (hipRTC) against the oracle, which
compiles the same source text as host C++ (needs an MI355X).  The FP64 path
must meet the 1e-12 bar, the FP32 path the FP32 bar, in both kernel layouts,
for several N (up to 16), M and constant vectors."""
import sys

import numpy as np
import pytest

from oracle import oracle as zo
from paper_1910_01965_amd import workloads as wl

import parity

pytestmark = pytest.mark.gpu

HEAD = "template <typename T> __device__ T integrand(const T* y, const T* x, const T* p) {\n"

# an oscillating, a peaked and a product integrand; p carries constants
WAVE = HEAD + ("  T s = p[1];\n  for (int k = 0; k < %d; ++k) s += (k + 1) * y[k];\n"
               "  return cos(x[0] * s) * exp(-p[0] * y[0] * y[0]) + p[2];\n}\n")
PEAK = HEAD + ("  T q = 0;\n  for (int k = 0; k < %d; ++k) { T d = y[k] - x[k %% %d]; q += d * d; }\n"
               "  return T(1) / (p[0] + q);\n}\n")
# the largest shape: all 16 parameters and 8 dimensions enter
SUM16 = HEAD + ("  T s = T(0);\n  for (int k = 0; k < 16; ++k) s += x[k];\n"
                "  for (int k = 0; k < 8; ++k) s += y[k];\n  return sin(s);\n}\n")
PRODUCT = HEAD + ("  T r = T(1);\n  for (int k = 0; k < %d; ++k) r *= T(1) + x[0] * sin(y[k]);\n"
                  "  return r;\n}\n")


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


def _cases(precision):
    out = []
    for N in (1, 3, 8, 12, 16):  # 12 and 16: the per-variant kernels of N > 8
        out.append(wl.ScanSpec("user", [np.linspace(0.2, 3, 9)], np.zeros(N), np.linspace(1, 2, N),
                               2051, 21, precision, name=f"wave N{N}", source=WAVE % N,
                               params=np.array([0.7, 0.3, 1.5])))
        M = min(3, N)
        out.append(wl.ScanSpec("user", [np.linspace(0.1, 0.9, 5)] * M, np.zeros(N), np.ones(N),
                               1024, 22, precision, name=f"peak N{N} M{M}", source=PEAK % (N, M),
                               params=np.array([0.2])))
    out.append(wl.ScanSpec("user", [np.linspace(-0.5, 0.5, 300)], np.zeros(4), np.ones(4), 4099, 23,
                           precision, name="product N4 G300", source=PRODUCT % 4))
    out.append(wl.ScanSpec("user", [], np.zeros(2), np.ones(2), 100003, 24, precision,
                           name="M0 one integral", source=WAVE.replace("x[0]", "T(2)") % 2,
                           params=np.array([1.0, 0.0, 0.0])))
    out.append(wl.ScanSpec("user", [np.array([0.0, 0.5 + k / 16.0]) for k in range(16)], np.zeros(8),
                           np.ones(8), 33, 25, precision, name="sum M16 N8", source=SUM16))
    return out


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("mode", ["point_major", "sample_major"])
def test_user_scans_match_oracle(precision, mode):
    import torch
    zmc = _zmc()
    for spec in _cases(precision):
        _say(f"user {spec.name} {precision} {mode}")
        f, s = zmc.scan(spec, mode=mode)
        torch.cuda.synchronize()
        f, s = f.cpu().numpy(), s.cpu().numpy()
        f_ref, s_ref = zo.scan(spec)
        _, _, msg = parity.check(f, s, f_ref, s_ref, spec.samples, precision, spec.name,
                                 small_n=spec.samples < 4096,
                                 volume=float(np.prod(spec.hi - spec.lo)))
        _say(msg)


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_user_values_match_oracle(precision):
    zmc = _zmc()
    for spec in _cases(precision)[:4]:
        for g in (0, spec.G - 1):
            got = zmc.debug_values(spec, g, 5, 70).cpu().numpy()
            ref = zo.values(spec, g, 5, 70)
            if precision == "fp64":
                assert np.allclose(got, ref, rtol=1e-13, atol=1e-14), (spec.name, g)
            else:
                assert np.all(np.abs(got - ref) <= 2e-5 * (1.0 + np.abs(ref))), (spec.name, g)


def test_fast_math_integrands():
    """ZMC_INTEGRAND_FAST_MATH: FP32 scans with approximate transcendentals and
    division meet the FP32 bar against the oracle in both layouts; the same
    handle's FP64 variants equal the accurate handle's bit for bit; and the
    FP32 results differ from the accurate handle's (the flag reaches the
    compiler)."""
    import torch
    zmc = _zmc()
    cases = [c for c in _cases("fp32") if c.name in ("wave N3", "peak N3 M3", "product N4 G300")]
    assert len(cases) == 3
    differ = 0
    for spec in cases:
        fast = spec.with_(fast_math=True)
        f_ref, s_ref = zo.scan(spec)
        for mode in ("point_major", "sample_major"):
            _say(f"fast-math user {spec.name} fp32 {mode}")
            f, s = zmc.scan(fast, mode=mode)
            fa, _ = zmc.scan(spec, mode=mode)
            torch.cuda.synchronize()
            f, s, fa = f.cpu().numpy(), s.cpu().numpy(), fa.cpu().numpy()
            _, _, msg = parity.check(f, s, f_ref, s_ref, spec.samples, "fp32", spec.name + " fast",
                                     small_n=spec.samples < 4096,
                                     volume=float(np.prod(spec.hi - spec.lo)))
            _say(msg)
            differ += int(not np.array_equal(f, fa))
        _say(f"fast-math user {spec.name} fp64")
        f64, s64 = zmc.scan(fast.with_(precision="fp64"))
        f64a, s64a = zmc.scan(spec.with_(precision="fp64"))
        torch.cuda.synchronize()
        assert torch.equal(f64, f64a) and torch.equal(s64, s64a), spec.name
    assert differ > 0


def test_user_splits_and_repeat_bitwise():
    import torch
    zmc = _zmc()
    spec = _cases("fp64")[2]                       # wave N3
    f_ref, s_ref = zo.scan(spec)
    outs = []
    for kw in (dict(mode="point_major", splits=1), dict(mode="point_major", splits=3),
               dict(mode="sample_major", splits=2), dict()):
        f, s = zmc.scan(spec, **kw)
        torch.cuda.synchronize()
        f, s = f.cpu().numpy(), s.cpu().numpy()
        parity.check(f, s, f_ref, s_ref, spec.samples, "fp64", f"wave N3 {kw}")
        outs.append((f, s))
    f2, s2 = zmc.scan(spec)
    torch.cuda.synchronize()
    assert np.array_equal(f2.cpu().numpy(), outs[-1][0]) and np.array_equal(s2.cpu().numpy(), outs[-1][1])


def test_user_reproduces_compiled_cosexp():
    """The COSEXP integrand written as a user function gives the compiled-in
    family's FP64 result to rounding."""
    import torch
    zmc = _zmc()
    src = HEAD + ("  T ph = x[0] * y[0] + x[1] * y[1];\n  for (int k = 2; k < 3; ++k) ph += y[k];\n"
                  "  return cos(ph) * exp(-(x[2] * x[2]) * y[0] * y[1]) + x[3];\n}\n")
    base = wl.cosexp_4p(points_per_axis=6, samples=4096, precision="fp64")
    base = base.with_(lo=np.zeros(3), hi=np.array([2.0, 1.0, 1.0]))
    user = base.with_(family="user", source=src)
    fa, sa = zmc.scan(base)
    fu, su = zmc.scan(user)
    torch.cuda.synchronize()
    fa, sa, fu, su = (t.cpu().numpy() for t in (fa, sa, fu, su))
    scale = np.maximum(np.abs(fa), sa * np.sqrt(base.samples))
    assert np.max(np.abs(fu - fa) / scale) < 1e-12 and np.max(np.abs(su - sa) / sa) < 1e-10


def test_user_integrand_shared_by_threads():
    """Threads sharing one handle compile and load its variants concurrently;
    every result equals the same scan run alone afterwards."""
    import threading

    import torch
    zmc = _zmc()
    src = HEAD + "  T s = p[0];\n  for (int k = 0; k < 2; ++k) s += x[0] * y[k];\n  return sin(s) + T(2);\n}\n"
    specs = [wl.ScanSpec("user", [np.linspace(0, 1, 37)], np.zeros(N), np.ones(N), 999, 50 + N, prec,
                         source=src, params=np.array([0.1]))
             for N in (2, 3, 4) for prec in ("fp64", "fp32")]
    out = [None] * len(specs)
    errors = []

    def run(i):
        try:
            f, s = zmc.scan(specs[i])
            torch.cuda.synchronize()
            out[i] = (f.cpu().numpy(), s.cpu().numpy())
        except Exception as e:  # reported below
            errors.append(e)

    th = [threading.Thread(target=run, args=(i,)) for i in range(len(specs))]
    for t in th:
        t.start()
    for t in th:
        t.join()
    assert not errors, errors
    for sp, (f, s) in zip(specs, out):
        fa, sa = zmc.scan(sp)
        torch.cuda.synchronize()
        assert np.array_equal(f, fa.cpu().numpy()) and np.array_equal(s, sa.cpu().numpy())


def _user_mix():
    wave = WAVE % 3
    peak = PEAK % (2, 2)
    out = []
    for i, prec in enumerate(("fp32", "fp64")):
        out.append(wl.ScanSpec("user", [np.linspace(0.2, 3, 40)], np.zeros(3), np.ones(3), 3001,
                               60 + i, prec, source=wave, params=np.array([0.7, 0.3, 1.5])))
        out.append(wl.ScanSpec("user", [np.linspace(0.1, 0.9, 30)] * 2, np.zeros(2), np.ones(2), 1024,
                               62 + i, prec, source=peak, params=np.array([0.2])))
        out.append(wl.gauss_2p(points_per_axis=50, samples=2048, precision=prec).with_(seed=64 + i))
    return out


def test_user_integrands_in_batches():
    """Batches mixing user integrands (their own run-time-built persistent
    kernels) with compiled-in families: graph replays and direct launches
    agree bitwise, each scan equals itself run alone, and the user scans
    meet the oracle bar."""
    import torch
    zmc = _zmc()
    specs = _user_mix()
    b = zmc.Batch(specs)
    assert b.info()["graph"] == 1
    runs = []
    for _ in range(2):
        b.launch()
        torch.cuda.synchronize()
        runs.append([(f.cpu().numpy(), s.cpu().numpy()) for f, s in b.outputs])
    b.close()
    direct = [(f.cpu().numpy(), s.cpu().numpy()) for f, s in zmc.scan_batch(specs, use_graph=False)]
    for i, sp in enumerate(specs):
        for other in (runs[1][i], direct[i]):
            assert np.array_equal(runs[0][i][0], other[0]) and np.array_equal(runs[0][i][1], other[1])
        fa, sa = zmc.scan_batch([sp])[0]
        assert np.array_equal(fa.cpu().numpy(), runs[0][i][0]), sp.name
        if sp.family == "user":
            f_ref, s_ref = zo.scan(sp)
            parity.check(runs[0][i][0], runs[0][i][1], f_ref, s_ref, sp.samples, sp.precision,
                         f"batched user {sp.precision}", small_n=sp.samples < 4096)


def test_user_integrands_in_the_server():
    import torch
    zmc = _zmc()
    specs = _user_mix()
    srv = zmc.Server(max_slots=4)
    tickets = [srv.submit(sp) for sp in specs]
    for t in tickets:
        assert srv.wait(t)[0] == 0
    torch.cuda.synchronize()
    for sp, t in zip(specs, tickets):
        f, s = srv.outputs(t)
        fa, sa = zmc.scan_batch([sp])[0]
        assert np.array_equal(f.cpu().numpy(), fa.cpu().numpy()), sp.name
        assert np.array_equal(s.cpu().numpy(), sa.cpu().numpy()), sp.name
    srv.close()


def test_a_variant_that_fails_to_compile_fails_alone():
    """An integrand that compiles only in FP64: a single FP32 scan fails with
    ZMC_E_INVALID and the compiler's message; in the server the FP32 request
    fails at admission while the other requests, the FP64 use of the same
    handle included, complete with their alone results; a batch holding it
    is refused as a whole; the library stays usable."""
    import torch
    zmc = _zmc()
    src = HEAD + '  static_assert(sizeof(T) == 8, "FP64 only");\n  return exp(-x[0] * y[0] * y[0]);\n}\n'
    ok64 = wl.ScanSpec("user", [np.linspace(0.5, 2.0, 30)], np.zeros(1), np.ones(1), 1024, 3, "fp64",
                       source=src)
    bad32 = ok64.with_(precision="fp32")
    with pytest.raises(zmc.ZmcError) as ei:
        zmc.scan(bad32)
    assert ei.value.status == 1 and "FP64 only" in str(ei.value)
    g32 = wl.gauss_2p(points_per_axis=40, samples=2048, precision="fp32")
    g64 = g32.with_(precision="fp64")
    srv = zmc.Server(max_slots=4)
    specs = [g32, bad32, ok64, g64]
    tickets = [srv.submit(sp) for sp in specs]
    assert [srv.wait(t)[0] for t in tickets] == [0, 1, 0, 0]
    torch.cuda.synchronize()
    for sp, t in zip(specs, tickets):
        if sp is bad32:
            continue
        f, s = srv.outputs(t)
        fa, sa = zmc.scan_batch([sp])[0]
        assert np.array_equal(f.cpu().numpy(), fa.cpu().numpy())
        assert np.array_equal(s.cpu().numpy(), sa.cpu().numpy())
    assert srv.stats()["failed"] == 1 and srv.stats()["completed"] == 3
    srv.close()
    with pytest.raises(zmc.ZmcError) as ei:
        zmc.Batch([g32, bad32])
    assert ei.value.status == 1
    f, s = zmc.scan(ok64)
    torch.cuda.synchronize()
    f_ref, s_ref = zo.scan(ok64)
    parity.check(f.cpu().numpy(), s.cpu().numpy(), f_ref, s_ref, ok64.samples, "fp64", "after failures")


@pytest.mark.parametrize("precision,fast_math", [("fp32", False), ("fp64", False), ("fp32", True)])
def test_user_gaussian_at_the_benchmark_size(precision, fast_math):
    """The Gaussian written as a user integrand on the full 1000 x 1000 grid
    with 2^14 samples, the configuration the benchmark times (FP32 also with
    approximate transcendentals): 300 sampled points and both corners against
    the oracle."""
    import torch
    zmc = _zmc()
    src = HEAD + "  return exp(-(x[0] * y[0] * y[0] + x[1] * y[1] * y[1] + y[2] * y[2]));\n}\n"
    spec = wl.gauss_2p(precision=precision).with_(family="user", source=src, fast_math=fast_math)
    _say(f"user gaussian 1e6 points {precision} fast_math={fast_math}")
    f, s = zmc.scan(spec)
    torch.cuda.synchronize()
    idx = np.sort(np.random.default_rng(2).choice(spec.G, 300, replace=False))
    idx = np.concatenate([[0, spec.G - 1], idx]).astype(np.uint64)
    ti = torch.from_numpy(idx.astype(np.int64)).cuda()
    fs, ss = f[ti].cpu().numpy(), s[ti].cpu().numpy()
    f_ref, s_ref = zo.scan(spec, idx)
    _, _, msg = parity.check(fs, ss, f_ref, s_ref, spec.samples, precision, "user gaussian 1e6")
    _say(msg)
