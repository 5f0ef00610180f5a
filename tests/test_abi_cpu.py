"""The C ABI on the CPU: the library loads, exports every declared symbol,
validates descriptors and plans work without touching a device."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_1910_01965_amd import zmc
from paper_1910_01965_amd import workloads as wl

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "zmc.h")


def _declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(zmc_[a-z_0-9]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(zmc.LIB_PATH):
        pytest.fail("libzmc.so is not built (run __graft_entry__.build())")
    return zmc.load()


def test_every_declared_symbol_is_exported(lib):
    names = _declared_functions()
    assert len(names) >= 9
    for name in names:
        assert hasattr(lib, name), name
    assert set(zmc.EXPORTS) == set(names)


def test_version(lib):
    assert lib.zmc_version().decode().startswith("zmc")


GOOD = wl.ScanSpec("gauss", [np.linspace(0.1, 10, 5), np.linspace(0.1, 10, 7)],
                   np.zeros(3), np.ones(3), 64, 1, "fp32")


@pytest.mark.parametrize("bad,status", [
    (GOOD.with_(samples=1), 1),
    (GOOD.with_(samples=0), 1),
    (GOOD.with_(lo=np.array([0.0, 1.0, 0.0])), 1),            # lo >= hi
    (GOOD.with_(hi=np.array([1.0, np.nan, 1.0])), 1),
    (GOOD.with_(lo=np.array([-np.inf, 0.0, 0.0])), 1),
    (GOOD.with_(family="cosexp"), 1),                          # needs M = 4
    (GOOD.with_(axes=[np.arange(1.0, 3.0)] * 4), 1),           # GAUSS needs M <= N
    (GOOD.with_(family="nope"), 1),
    (GOOD.with_(precision="fp16"), 1),
    (GOOD.with_(axes=[np.zeros(0), np.linspace(0.1, 10, 7)]), 1),  # an empty axis (G = 0)
    (GOOD.with_(axes=[np.arange(2.0)] * 17), 1),               # M > 16
    (GOOD.with_(lo=np.zeros(17), hi=np.ones(17)), 1),          # N > 16
    (GOOD.with_(axes=[np.arange(1 << 21, dtype=np.float64)] * 3, family="sin_sum"), 1),  # G > 2^62
])
def test_invalid_descriptors(lib, bad, status):
    with pytest.raises(zmc.ZmcError) as ei:
        zmc.validate(bad)
    assert ei.value.status == status
    assert lib.zmc_last_error().decode() != ""


def test_valid_descriptors(lib):
    assert zmc.validate(GOOD) == 35
    assert zmc.validate(wl.ScanSpec("sin_sum", [], np.zeros(2), np.ones(2), 2, 0)) == 1
    assert zmc.validate(wl.plain_fp64()) == 1000
    assert zmc.validate(wl.gauss_2p()) == 10**6
    assert zmc.validate(wl.cosexp_4p()) == 10**8
    for N in (9, 12, 16):  # every N up to 16 is built
        assert zmc.validate(GOOD.with_(lo=np.zeros(N), hi=np.ones(N))) == 35
    assert lib.zmc_last_error().decode() == ""


def test_null_descriptor_and_outputs(lib):
    assert lib.zmc_validate(None, None) == 1
    d = zmc.Desc(GOOD)
    assert lib.zmc_scan(d.ref, None, None) == 1
    assert lib.zmc_scan_device(d.ref, None, None, None, None) == 1
    # no device lists and no host lists either, with M > 0
    d.c.axis_vals = None
    fake = ctypes.c_void_p(0x1000)                  # never dereferenced: refused first
    assert lib.zmc_scan_device(d.ref, None, fake, fake, None) == 1
    assert "both NULL" in lib.zmc_last_error().decode()
    assert lib.zmc_debug_words(0, 0, 0, -1, None, None) == 1
    assert lib.zmc_debug_words(0, 0, 0, 4, None, None) == 1


def _covers(p):
    # the pieces cover every group exactly once, none empty
    assert p["splits"] >= 1
    assert p["splits"] * p["groups_per_split"] >= p["groups"]
    assert (p["splits"] - 1) * p["groups_per_split"] < p["groups"]


@pytest.mark.parametrize("spec", [wl.plain_fp64(), wl.gauss_2p(), wl.cosexp_4p(),
                                  wl.plain_fp64(points=3, samples=7),
                                  wl.gauss_2p(points_per_axis=9, samples=4097)])
def test_plans_cover_all_work(lib, spec):
    for mode in ("auto", "point_major", "sample_major"):
        # explicit splits up to and past the group count (ragged sample
        # counts included): the planner never leaves a piece empty
        for splits in (None, 1, 3, 1000, 1024, 1025, 4097, 65535):
            p = zmc.plan(spec, mode=mode, splits=splits, cu_count=256)
            _covers(p)
            assert p["grid_points"] == spec.G
            assert p["groups"] == (spec.samples + 3) // 4
            if p["splits"] > 1:
                assert p["workspace_bytes"] == 16 * p["splits"] * spec.G
            else:
                assert p["workspace_bytes"] == 0


def test_auto_plans_for_the_workloads(lib):
    p0 = zmc.plan(wl.plain_fp64(), cu_count=256)
    assert p0["mode"] == "sample_major"
    p1 = zmc.plan(wl.gauss_2p(), cu_count=256)
    assert p1["mode"] == "point_major" and p1["splits"] > 1
    p2 = zmc.plan(wl.cosexp_4p(), cu_count=256)
    assert p2["mode"] == "point_major" and p2["splits"] == 1 and p2["blocks"] == 390625


def test_bad_launch_options(lib):
    for kw in ({"block": 100}, {"block": 2048}, {"mode": "point_major", "block": 512}):
        with pytest.raises(zmc.ZmcError):
            zmc.plan(GOOD, cu_count=256, **kw)


def test_batch_plan_on_cpu(lib):
    specs = wl.batched_512()
    info = zmc.batch_plan(specs, cu_count=256)
    assert info["scans"] == 512 and 1 <= info["variants"] <= 21
    assert info["points"] == sum(s.G for s in specs)
    assert info["samples"] == sum(s.G * s.samples for s in specs)
    # tile count: point-major tiles of 256 points x ceil(groups / pm_groups) pieces
    one = [wl.gauss_2p(points_per_axis=100, samples=10_000)]
    p = zmc.batch_plan(one, cu_count=256, pm_groups=100, pm_min_points=1)
    assert p["tiles"] == ((10_000 // 256) + 1) * 25 and p["merge_scans"] == 1
    p = zmc.batch_plan(one, cu_count=256, pm_groups=10_000, pm_min_points=1)
    assert p["tiles"] == (10_000 // 256) + 1 and p["merge_scans"] == 0
    # grids below the point-major threshold: one tile per point and piece
    p = zmc.batch_plan(one, cu_count=256, pm_min_points=10_001, sm_groups=1000)
    assert p["tiles"] == 10_000 * 3 and p["merge_scans"] == 1
    p = zmc.batch_plan(one, cu_count=256, pm_min_points=10**9, sm_groups=625)
    assert p["tiles"] == 10_000 * 4


def test_batch_plan_names_the_bad_scan(lib):
    specs = wl.batched_512()[:5]
    specs[3] = specs[3].with_(samples=1)
    with pytest.raises(zmc.ZmcError) as ei:
        zmc.batch_plan(specs, cu_count=256)
    assert ei.value.status == 1 and "scan 3" in str(ei.value)
    with pytest.raises(zmc.ZmcError):
        zmc.batch_plan([], cu_count=256)


USER_SRC = ("template <typename T> __device__ T integrand(const T* y, const T* x, const T* p) {\n"
            "  return sin(x[0] * y[0]) * exp(-p[0] * y[1] * y[1]) + p[1];\n}\n")


def test_user_integrand_compiles_without_a_gpu(lib):
    it = zmc.Integrand(USER_SRC)
    assert it.handle
    spec = wl.ScanSpec("user", [np.linspace(0, 1, 5)], np.zeros(2), np.ones(2), 100, 3, "fp32",
                       source=USER_SRC, params=np.array([0.5, 2.0]))
    assert zmc.validate(spec) == 5
    it.close()


def test_user_integrand_compile_error_is_reported(lib):
    bad = USER_SRC.replace("exp(", "no_such_function(")
    with pytest.raises(zmc.ZmcError) as ei:
        zmc.Integrand(bad)
    assert ei.value.status == 1 and "no_such_function" in str(ei.value)
    with pytest.raises(zmc.ZmcError):
        zmc.Integrand("")


def test_user_descriptor_validation(lib):
    spec = wl.ScanSpec("user", [np.linspace(0, 1, 5)], np.zeros(2), np.ones(2), 100, 3,
                       source=USER_SRC, params=np.zeros(17))
    with pytest.raises(zmc.ZmcError) as ei:
        zmc.validate(spec)                        # more than 16 constants
    assert ei.value.status == 1
    with pytest.raises(zmc.ZmcError):
        zmc.validate(spec.with_(params=np.array([np.inf])))
    d = zmc.Desc(spec.with_(params=np.zeros(2)))
    d.c.integrand = None                          # ZMC_USER without a handle
    G = ctypes_u64()
    assert lib.zmc_validate(d.ref, G) == 1
    # built-in families take no constants
    with pytest.raises(zmc.ZmcError):
        zmc.validate(GOOD.with_(params=np.ones(1)))


def test_user_scans_plan_as_their_own_variants(lib):
    spec = wl.ScanSpec("user", [np.linspace(0, 1, 5)], np.zeros(2), np.ones(2), 100, 3,
                       source=USER_SRC, params=np.array([0.5, 2.0]))
    info = zmc.batch_plan([GOOD, spec, spec.with_(seed=4)], cu_count=256)
    assert info["scans"] == 3 and info["variants"] == 2
    # another shape of the same integrand is another kernel; one_kernel keeps it apart
    info = zmc.batch_plan([GOOD, spec, spec.with_(axes=[np.arange(3.0)] * 2)], cu_count=256,
                          one_kernel=1)
    assert info["variants"] == 3


def ctypes_u64():
    import ctypes
    return ctypes.byref(ctypes.c_uint64())


def test_chunked_scan_argument_checks(lib):
    import ctypes
    d = zmc.Desc(GOOD)
    f = np.zeros(GOOD.G)
    s = np.zeros(GOOD.G)
    vp = ctypes.c_void_p
    assert lib.zmc_scan_chunked(d.ref, None, vp(s.ctypes.data), 0) == 1
    assert lib.zmc_scan_chunked(d.ref, vp(f.ctypes.data), None, 0) == 1
    bad = zmc.Desc(GOOD.with_(samples=1))
    assert lib.zmc_scan_chunked(bad.ref, vp(f.ctypes.data), vp(s.ctypes.data), 0) == 1
    no_lists = zmc.Desc(GOOD)
    no_lists.c.axis_vals = None
    assert lib.zmc_scan_chunked(no_lists.ref, vp(f.ctypes.data), vp(s.ctypes.data), 0) == 1
    # a valid request on a host without a GPU fails cleanly (no device)
    import torch
    if not torch.cuda.is_available():
        assert lib.zmc_scan_chunked(d.ref, vp(f.ctypes.data), vp(s.ctypes.data), 7) == 3
        assert lib.zmc_last_error().decode()


def test_range_scan_argument_checks(lib):
    import ctypes
    d = zmc.Desc(GOOD)
    f = np.zeros(GOOD.G)
    vp = ctypes.c_void_p
    assert lib.zmc_scan_range(d.ref, 3, 3, vp(f.ctypes.data), vp(f.ctypes.data), 0) == 1
    assert lib.zmc_scan_range(d.ref, 0, GOOD.G + 1, vp(f.ctypes.data), vp(f.ctypes.data), 0) == 1
    assert lib.zmc_scan_range(d.ref, 4, 2, vp(f.ctypes.data), vp(f.ctypes.data), 0) == 1


def test_binding_fails_loudly_without_the_library(monkeypatch):
    # no CPU fallback: every entry point of the binding needs the HIP library
    monkeypatch.setattr(zmc, "_lib", None)
    monkeypatch.setattr(zmc, "LIB_PATH", "/nonexistent/libzmc.so")
    spec = wl.gauss_2p(points_per_axis=4, samples=8)
    for call in (lambda: zmc.scan(spec), lambda: zmc.scan_host(spec), lambda: zmc.plan(spec),
                 lambda: zmc.scan_chunked(spec), lambda: zmc.Batch([spec]), lambda: zmc.Server()):
        with pytest.raises(RuntimeError, match="no fallback"):
            call()


def test_oversized_buffers_are_refused_before_any_device_call(lib):
    # sizes that would wrap 2^64 if formed: refused with ZMC_E_NOMEM before
    # any HIP call (on a machine without a GPU a HIP call would give
    # ZMC_E_DEVICE instead)
    big = wl.ScanSpec("sin_sum", [np.arange(2.0 ** 19)] * 3, np.zeros(2), np.ones(2), 1 << 20, 1,
                      "fp32")                                        # G = 2^57
    with pytest.raises(zmc.ZmcError) as ei:
        zmc.plan(big, mode="point_major", splits=65535, cu_count=256)
    assert ei.value.status == 2 and "split partials" in str(ei.value)
    d = zmc.Desc(big)
    f = np.zeros(4)
    dp = ctypes.POINTER(ctypes.c_double)
    assert lib.zmc_scan(d.ref, f.ctypes.data_as(dp), f.ctypes.data_as(dp)) == 2
    assert "staging" in lib.zmc_last_error().decode()
    st = lib.zmc_scan_range(d.ref, 0, 1 << 56, ctypes.c_void_p(f.ctypes.data),
                            ctypes.c_void_p(f.ctypes.data), 1 << 56)
    assert st == 2 and "chunks" in lib.zmc_last_error().decode()


def test_integrate_front_end_rejects_bad_arguments(lib):
    # checked by the library before any device use
    with pytest.raises(zmc.ZmcError) as ei:
        zmc.integrate("gauss", [(1.0, 0.0)] * 3, [[1.0, 2.0]], 64)      # lo >= hi
    assert ei.value.status == 1
    with pytest.raises(zmc.ZmcError) as ei:
        zmc.integrate("not a function", [(0.0, 1.0)], [[1.0]], 64)     # source that does not compile
    assert ei.value.status == 1


def test_log_level_from_the_environment():
    # ZMC_LOG=2 reports plans and set-up on stderr; unset, the library is silent
    import subprocess
    import sys
    code = ("from paper_1910_01965_amd import zmc, workloads as wl\n"
            "zmc.plan(wl.gauss_2p(), cu_count=256)\n"
            "zmc.batch_plan(wl.batched_512()[:2], cu_count=256)\n")
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    env = {k: v for k, v in os.environ.items() if k != "ZMC_LOG"}
    quiet = subprocess.run([sys.executable, "-c", code], cwd=root, env=env, capture_output=True,
                           text=True, timeout=120)
    assert quiet.returncode == 0 and "[zmc]" not in quiet.stderr
    loud = subprocess.run([sys.executable, "-c", code], cwd=root, env=dict(env, ZMC_LOG="2"),
                          capture_output=True, text=True, timeout=120)
    assert loud.returncode == 0
    assert "[zmc] plan: G=1000000 n=16384 N=3 point-major" in loud.stderr
    assert "[zmc] tune table" in loud.stderr


def test_c_program_uses_the_abi_without_python():
    # tests/c/zmc_abi_check.c: include/zmc.h and libzmc.so from plain C
    import subprocess
    exe = os.path.join(os.path.dirname(os.path.abspath(__file__)), "c", "zmc_abi_check")
    if not os.path.exists(exe):
        pytest.fail("tests/c/zmc_abi_check is not built (run __graft_entry__.build())")
    r = subprocess.run([exe], capture_output=True, text=True, timeout=60)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "passed (host-only part)" in r.stdout
    # the Python binding's structures have the C layouts
    import ctypes as ct
    sizes = dict(zip(*[iter(next(ln for ln in r.stdout.splitlines()
                                  if ln.startswith("sizeof:")).split()[1:])] * 2))
    assert int(sizes["scan_desc"]) == ct.sizeof(zmc.ScanDesc)
    assert int(sizes["launch_opts"]) == ct.sizeof(zmc.LaunchOpts)
    assert int(sizes["plan_info"]) == ct.sizeof(zmc.PlanInfo)
    assert int(sizes["batch_opts"]) == ct.sizeof(zmc.BatchOpts)
    assert int(sizes["batch_info"]) == ct.sizeof(zmc.BatchInfo)
    assert int(sizes["server_opts"]) == ct.sizeof(zmc.ServerOpts)
    assert int(sizes["server_stats"]) == ct.sizeof(zmc.ServerStats)


def test_server_rejects_bad_admission_options(lib):
    # checked before any device call, so this runs without a GPU
    out = ctypes.c_void_p()
    for admission, max_wait in ((2, 0), (-1, 0), (1, -5)):
        o = zmc.ServerOpts(0, 0, 0, 0, 0, 0, admission, max_wait)
        assert lib.zmc_server_create(ctypes.byref(o), ctypes.byref(out)) == 1
        assert b"admission" in lib.zmc_last_error()
        assert not out.value
    o = zmc.ServerOpts(0, 0, 0, 0, 0, 0, 0, 0, -1)
    assert lib.zmc_server_create(ctypes.byref(o), ctypes.byref(out)) == 1
    assert b"slice_us" in lib.zmc_last_error()
    assert not out.value


def test_tune_table_source():
    # the tile table next to libzmc.so by default; ZMC_TUNE_TABLE overrides it,
    # and a missing file falls back to the built-in shapes (host only)
    import subprocess
    import sys
    code = "from paper_1910_01965_amd import zmc\nprint(zmc.tune_source())\n"
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    env = {k: v for k, v in os.environ.items() if k != "ZMC_TUNE_TABLE"}
    runs = {}
    for name, extra in (("default", {}), ("missing", {"ZMC_TUNE_TABLE": "/nonexistent/t.txt"})):
        r = subprocess.run([sys.executable, "-c", code], cwd=root, env=dict(env, **extra),
                           capture_output=True, text=True, timeout=120)
        assert r.returncode == 0, r.stderr
        runs[name] = r.stdout.strip()
    expected = os.path.join(os.path.dirname(zmc.LIB_PATH), "tune_table.txt")
    assert os.path.realpath(runs["default"]) == os.path.realpath(expected)
    assert runs["missing"] == "built-in defaults"


def test_wide_scans_take_at_most_256_threads_per_block(lib):
    """N > 8: sample-major blocks of more than 256 threads are refused (their
    kernels are built for 256), host-only with an explicit CU count."""
    sp = GOOD.with_(lo=np.zeros(12), hi=np.ones(12))
    with pytest.raises(zmc.ZmcError) as ei:
        zmc.plan(sp, mode="sample_major", block=512, cu_count=256)
    assert ei.value.status == 1 and "256" in str(ei.value)
    assert zmc.plan(sp, mode="sample_major", block=256, cu_count=256)["block"] == 256
    assert zmc.plan(GOOD, mode="sample_major", block=1024, cu_count=256)["block"] == 1024


def test_fast_math_integrand_compiles_without_a_gpu(lib):
    it = zmc.Integrand(USER_SRC, fast_math=True)   # compiles an FP64 and an FP32 variant
    assert it.handle and it.fast_math
    it.close()
    h = ctypes.c_void_p()
    assert lib.zmc_integrand_create_ex(USER_SRC.encode(), ctypes.c_uint32(2), ctypes.byref(h)) == 1
    assert "unknown flags" in lib.zmc_last_error().decode() and not h.value
    # process-wide handles are per (source, mode)
    assert zmc.integrand(USER_SRC) is not zmc.integrand(USER_SRC, fast_math=True)
    assert zmc.integrand(USER_SRC, fast_math=True) is zmc.integrand(USER_SRC, fast_math=True)
