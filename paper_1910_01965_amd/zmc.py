"""Python binding of libzmc (include/zmc.h): argument marshalling only.

Every step of the scan runs in the HIP library; this module converts a
`ScanSpec` (see workloads.py) into the C descriptor, hands torch device
buffers and streams to the library, and raises on a non-zero status.  It
fails loudly when libzmc.so has not been built: there is no fallback.
"""
import ctypes
import os
import threading

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libzmc.so")

FAMILY = {"sin_sum": 0, "gauss": 1, "cosexp": 2, "const": 3, "linear": 4, "user": 5}
PRECISION = {"fp64": 0, "fp32": 1}
MODE = {"auto": 0, "point_major": 1, "sample_major": 2}
MODE_NAME = {v: k for k, v in MODE.items()}
STATUS = {0: "ZMC_OK", 1: "ZMC_E_INVALID", 2: "ZMC_E_NOMEM", 3: "ZMC_E_DEVICE",
          4: "ZMC_E_UNSUPPORTED", 5: "ZMC_E_BUSY", 6: "ZMC_E_CANCELLED"}

EXPORTS = ("zmc_last_error", "zmc_version", "zmc_validate", "zmc_plan", "zmc_scan",
           "zmc_scan_device", "zmc_scan_device_ex", "zmc_scan_device_noalloc", "zmc_debug_words",
           "zmc_debug_values",
           "zmc_batch_default_opts", "zmc_batch_plan", "zmc_batch_create", "zmc_batch_launch",
           "zmc_batch_get_info", "zmc_batch_destroy", "zmc_scan_batch", "zmc_tune_source",
           "zmc_server_create", "zmc_server_submit", "zmc_server_poll", "zmc_server_wait",
           "zmc_server_get_stats", "zmc_server_release", "zmc_server_cancel", "zmc_server_destroy",
           "zmc_integrand_create", "zmc_integrand_create_ex",
           "zmc_integrand_log", "zmc_integrand_destroy", "zmc_scan_chunked", "zmc_scan_range",
           "zmc_debug_valu_probe", "zmc_debug_rate_probe")


class ZmcError(RuntimeError):
    def __init__(self, status, message):
        super().__init__(f"{STATUS.get(status, status)}: {message}")
        self.status = status


class ScanDesc(ctypes.Structure):
    _fields_ = [
        ("M", ctypes.c_int32),
        ("N", ctypes.c_int32),
        ("axis_len", ctypes.POINTER(ctypes.c_int64)),
        ("axis_vals", ctypes.POINTER(ctypes.c_double)),
        ("lo", ctypes.POINTER(ctypes.c_double)),
        ("hi", ctypes.POINTER(ctypes.c_double)),
        ("family", ctypes.c_int32),
        ("precision", ctypes.c_int32),
        ("params", ctypes.POINTER(ctypes.c_double)),
        ("n_params", ctypes.c_int32),
        ("samples", ctypes.c_uint64),
        ("seed", ctypes.c_uint64),
        ("integrand", ctypes.c_void_p),
    ]


class LaunchOpts(ctypes.Structure):
    _fields_ = [("mode", ctypes.c_int32), ("block", ctypes.c_int32),
                ("splits", ctypes.c_int32), ("cu_count", ctypes.c_int32),
                ("ev_begin", ctypes.c_void_p), ("ev_end", ctypes.c_void_p)]


class PlanInfo(ctypes.Structure):
    _fields_ = [("mode", ctypes.c_int32), ("block", ctypes.c_int32),
                ("splits", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("grid_points", ctypes.c_uint64), ("groups", ctypes.c_uint64),
                ("groups_per_split", ctypes.c_uint64), ("blocks", ctypes.c_uint64),
                ("workspace_bytes", ctypes.c_uint64)]


class BatchOpts(ctypes.Structure):
    _fields_ = [("use_graph", ctypes.c_int32), ("parallel_variants", ctypes.c_int32),
                ("pm_groups", ctypes.c_int64), ("sm_groups", ctypes.c_int64),
                ("pm_min_points", ctypes.c_int64), ("cu_count", ctypes.c_int32),
                ("one_kernel", ctypes.c_int32)]


class BatchInfo(ctypes.Structure):
    _fields_ = [("scans", ctypes.c_int32), ("variants", ctypes.c_int32), ("tiles", ctypes.c_int64),
                ("samples", ctypes.c_uint64), ("points", ctypes.c_uint64),
                ("workspace_bytes", ctypes.c_uint64), ("merge_scans", ctypes.c_int32),
                ("graph", ctypes.c_int32)]


class ServerOpts(ctypes.Structure):
    _fields_ = [("hbm_budget_bytes", ctypes.c_uint64), ("max_slots", ctypes.c_int32),
                ("slice_tiles", ctypes.c_int32), ("max_inflight", ctypes.c_int32),
                ("cu_count", ctypes.c_int32), ("slice_samples", ctypes.c_uint64),
                ("admission", ctypes.c_int32), ("max_wait_ms", ctypes.c_int32),
                ("slice_us", ctypes.c_int32)]

ADMISSION = {"fifo": 0, "shortest": 1}


class ServerStats(ctypes.Structure):
    _fields_ = [(k, ctypes.c_uint64) for k in (
        "submitted", "admitted", "completed", "failed", "pending", "active", "samples_completed",
        "slices", "tiles", "bytes_in_use", "bytes_peak")] + [
        (k, ctypes.c_double) for k in ("latency_p50_s", "latency_p99_s", "latency_max_s",
                                       "samples_per_s")] + [("tickets", ctypes.c_uint64),
                                                            ("slice_samples_now", ctypes.c_uint64),
                                                            ("cancelled", ctypes.c_uint64)]


_lib = None


def load():
    """The loaded libzmc (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                               "`python -m paper_1910_01965_amd.build` (no fallback exists)")
        lib = ctypes.CDLL(LIB_PATH)
        vp = ctypes.c_void_p
        dp = ctypes.POINTER(ctypes.c_double)
        descp = ctypes.POINTER(ScanDesc)
        lib.zmc_last_error.restype = ctypes.c_char_p
        lib.zmc_version.restype = ctypes.c_char_p
        lib.zmc_validate.argtypes = [descp, ctypes.POINTER(ctypes.c_uint64)]
        lib.zmc_plan.argtypes = [descp, ctypes.POINTER(LaunchOpts), ctypes.POINTER(PlanInfo)]
        lib.zmc_scan.argtypes = [descp, dp, dp]
        lib.zmc_scan_chunked.argtypes = [descp, vp, vp, ctypes.c_uint64]
        lib.zmc_scan_range.argtypes = [descp, ctypes.c_uint64, ctypes.c_uint64, vp, vp, ctypes.c_uint64]
        lib.zmc_scan_device.argtypes = [descp, vp, vp, vp, vp]
        lib.zmc_scan_device_ex.argtypes = [descp, vp, vp, vp, ctypes.POINTER(LaunchOpts), vp]
        lib.zmc_scan_device_noalloc.argtypes = [descp, vp, vp, vp, vp]
        lib.zmc_debug_words.argtypes = [ctypes.c_uint64, ctypes.c_uint64, ctypes.c_uint64,
                                        ctypes.c_int64, vp, vp]
        lib.zmc_debug_values.argtypes = [descp, vp, ctypes.c_uint64, ctypes.c_uint64,
                                         ctypes.c_int64, vp, vp]
        lib.zmc_debug_valu_probe.argtypes = [ctypes.c_int32, ctypes.c_int64, vp, vp]
        lib.zmc_debug_rate_probe.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_int64, vp, vp]
        ptrs = ctypes.POINTER(ctypes.c_void_p)
        lib.zmc_batch_default_opts.argtypes = [ctypes.POINTER(BatchOpts)]
        lib.zmc_batch_default_opts.restype = None
        lib.zmc_batch_plan.argtypes = [descp, ctypes.c_int32, ctypes.POINTER(BatchOpts),
                                       ctypes.POINTER(BatchInfo)]
        lib.zmc_batch_create.argtypes = [descp, ctypes.c_int32, ptrs, ptrs, ptrs,
                                         ctypes.POINTER(BatchOpts), ctypes.POINTER(vp)]
        lib.zmc_batch_launch.argtypes = [vp, vp]
        lib.zmc_batch_get_info.argtypes = [vp, ctypes.POINTER(BatchInfo)]
        lib.zmc_batch_destroy.argtypes = [vp]
        lib.zmc_scan_batch.argtypes = [descp, ctypes.c_int32, ptrs, ptrs, ptrs, vp]
        lib.zmc_tune_source.restype = ctypes.c_char_p
        u64p = ctypes.POINTER(ctypes.c_uint64)
        lib.zmc_server_create.argtypes = [ctypes.POINTER(ServerOpts), ctypes.POINTER(vp)]
        lib.zmc_server_submit.argtypes = [vp, descp, vp, vp, vp, u64p]
        lib.zmc_server_poll.argtypes = [vp, ctypes.c_uint64, ctypes.POINTER(ctypes.c_int32),
                                        ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_double)]
        lib.zmc_server_wait.argtypes = [vp, ctypes.c_uint64, ctypes.POINTER(ctypes.c_int),
                                        ctypes.POINTER(ctypes.c_double)]
        lib.zmc_server_get_stats.argtypes = [vp, ctypes.POINTER(ServerStats)]
        lib.zmc_server_release.argtypes = [vp, ctypes.c_uint64]
        lib.zmc_server_cancel.argtypes = [vp, ctypes.c_uint64]
        lib.zmc_server_destroy.argtypes = [vp]
        lib.zmc_integrand_create.argtypes = [ctypes.c_char_p, ctypes.POINTER(vp)]
        lib.zmc_integrand_create_ex.argtypes = [ctypes.c_char_p, ctypes.c_uint32, ctypes.POINTER(vp)]
        lib.zmc_integrand_log.argtypes = [vp]
        lib.zmc_integrand_log.restype = ctypes.c_char_p
        lib.zmc_integrand_destroy.argtypes = [vp]
        for name in ("zmc_integrand_create", "zmc_integrand_create_ex", "zmc_integrand_destroy",
                     "zmc_scan_chunked",
                     "zmc_scan_range",
                     "zmc_validate", "zmc_plan", "zmc_scan", "zmc_scan_device",
                     "zmc_scan_device_ex", "zmc_scan_device_noalloc", "zmc_debug_words", "zmc_debug_values",
                     "zmc_batch_plan", "zmc_batch_create", "zmc_batch_launch",
                     "zmc_batch_get_info", "zmc_batch_destroy", "zmc_scan_batch",
                     "zmc_server_create", "zmc_server_submit", "zmc_server_poll",
                     "zmc_server_wait", "zmc_server_get_stats", "zmc_server_release",
                     "zmc_server_cancel", "zmc_server_destroy"):
            getattr(lib, name).restype = ctypes.c_int
        _lib = lib
    return _lib


def _check(status):
    if status != 0:
        raise ZmcError(status, load().zmc_last_error().decode())


INTEGRAND_FAST_MATH = 1


class Integrand:
    """A user integrand compiled at run time (zmc_integrand_create_ex): `source`
    defines template <typename T> __device__ T integrand(const T* y,
    const T* x, const T* p).  `fast_math`: FP32 variants use approximate
    transcendentals (ZMC_INTEGRAND_FAST_MATH).  Raises ZmcError (with the
    compiler's log) when it does not compile."""

    def __init__(self, source, fast_math=False):
        lib = load()
        h = ctypes.c_void_p()
        flags = INTEGRAND_FAST_MATH if fast_math else 0
        _check(lib.zmc_integrand_create_ex(source.encode(), ctypes.c_uint32(flags), ctypes.byref(h)))
        self.source = source
        self.fast_math = bool(fast_math)
        self.handle = h.value
        self._lib = lib

    def log(self):
        return self._lib.zmc_integrand_log(ctypes.c_void_p(self.handle)).decode()

    def close(self):
        if self.handle:
            _check(self._lib.zmc_integrand_destroy(ctypes.c_void_p(self.handle)))
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


_integrands = {}
_integrands_lock = threading.Lock()


def integrand(source, fast_math=False):
    """The process-wide Integrand for (`source`, `fast_math`) (compiled once,
    kept for the life of the process, so its kernels are never unloaded under
    a scan)."""
    if not source:
        raise ZmcError(1, "family 'user' needs ScanSpec.source")
    key = (source, bool(fast_math))
    with _integrands_lock:
        it = _integrands.get(key)
        if it is None:
            it = _integrands[key] = Integrand(source, fast_math)
    return it


class Desc:
    """A C descriptor for one ScanSpec; keeps its host arrays alive."""

    def __init__(self, spec, precision=None):
        self.spec = spec
        self.axis_len = np.array([len(a) for a in spec.axes], dtype=np.int64)
        self.axis_vals = (np.concatenate(spec.axes) if spec.axes else np.zeros(1)).astype(np.float64)
        self.lo = np.ascontiguousarray(spec.lo, dtype=np.float64)
        self.hi = np.ascontiguousarray(spec.hi, dtype=np.float64)
        prec = precision or spec.precision
        self.params = np.ascontiguousarray(getattr(spec, "params", np.zeros(0)), dtype=np.float64)
        self.integrand = integrand(spec.source, getattr(spec, "fast_math", False)) \
            if spec.family == "user" else None
        self.c = ScanDesc(
            M=len(spec.axes), N=len(self.lo),
            axis_len=self.axis_len.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
            axis_vals=self.axis_vals.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
            lo=self.lo.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
            hi=self.hi.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
            family=FAMILY.get(spec.family, -1), precision=PRECISION.get(prec, -1),
            params=self.params.ctypes.data_as(ctypes.POINTER(ctypes.c_double)) if self.params.size else None,
            n_params=int(self.params.size), samples=int(spec.samples),
            seed=int(spec.seed) & 0xFFFFFFFFFFFFFFFF,
            integrand=self.integrand.handle if self.integrand is not None else None)

    @property
    def ref(self):
        return ctypes.byref(self.c)


def _opts(mode=None, block=None, splits=None, cu_count=None, events=None):
    if mode is None and block is None and splits is None and cu_count is None and events is None:
        return None
    ev_b, ev_e = events if events is not None else (None, None)
    return LaunchOpts(MODE[mode or "auto"], int(block or 0), int(splits or 0), int(cu_count or 0),
                      ev_b, ev_e)


def validate(spec):
    """Grid size G of a valid spec (raises ZmcError otherwise)."""
    G = ctypes.c_uint64()
    d = Desc(spec)
    _check(load().zmc_validate(d.ref, ctypes.byref(G)))
    return G.value


def plan(spec, mode=None, block=None, splits=None, cu_count=None):
    """The work decomposition the library would use, as a dict."""
    o = _opts(mode, block, splits, cu_count)
    info = PlanInfo()
    desc = Desc(spec)
    _check(load().zmc_plan(desc.ref, ctypes.byref(o) if o else None, ctypes.byref(info)))
    out = {k: getattr(info, k) for k, _ in PlanInfo._fields_ if k != "reserved"}
    out["mode"] = MODE_NAME.get(out["mode"], out["mode"])
    return out


def _stream_ptr(stream):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def axis_tensor(spec, device="cuda"):
    """The concatenated parameter lists as a float64 device tensor."""
    import torch
    vals = np.concatenate(spec.axes) if spec.axes else np.zeros(1)
    return torch.from_numpy(np.ascontiguousarray(vals, dtype=np.float64)).to(device)


def scan_device(spec, d_axis, f, sigma, stream=None, mode=None, block=None, splits=None,
                events=None):
    """Enqueue the scan of `spec` on `stream`; f and sigma are float64 device
    tensors of G elements; d_axis holds the parameter lists on the device
    (None: the library stages them from the spec for this call).  `events` =
    (begin, end) raw hipEvent_t handles recorded around the main kernel."""
    o = _opts(mode, block, splits, events=events)
    d = Desc(spec)
    _check(load().zmc_scan_device_ex(d.ref, ctypes.c_void_p(d_axis.data_ptr() if d_axis is not None else None),
                                     ctypes.c_void_p(f.data_ptr()), ctypes.c_void_p(sigma.data_ptr()),
                                     ctypes.byref(o) if o else None, _stream_ptr(stream)))


def scan_device_noalloc(spec, d_axis, f, sigma, stream=None):
    """Enqueue the scan of `spec` through the allocation-free entry point:
    the plan and results of scan_device, with the split partials in the
    library's fixed per-device scratch (ZmcError with status 2 when they do
    not fit it)."""
    d = Desc(spec)
    _check(load().zmc_scan_device_noalloc(d.ref, ctypes.c_void_p(d_axis.data_ptr()),
                                          ctypes.c_void_p(f.data_ptr()),
                                          ctypes.c_void_p(sigma.data_ptr()), _stream_ptr(stream)))


NOALLOC_SCRATCH_BYTES = 128 << 20  # ZMC_NOALLOC_SCRATCH_BYTES of include/zmc.h


def scan(spec, mode=None, block=None, splits=None, stream=None):
    """(f, sigma) float64 device tensors for every grid point of `spec`,
    allocated on and computed on `stream` (default: the current stream)."""
    import torch
    G = validate(spec)
    with torch.cuda.stream(stream if stream is not None else torch.cuda.current_stream()):
        d_axis = axis_tensor(spec)
        f = torch.empty(G, dtype=torch.float64, device="cuda")
        s = torch.empty(G, dtype=torch.float64, device="cuda")
    scan_device(spec, d_axis, f, s, stream=stream, mode=mode, block=block, splits=splits)
    return f, s


def scan_host(spec):
    """(f, sigma) numpy arrays through the synchronous host-memory entry point."""
    d = Desc(spec)
    G = validate(spec)
    f = np.empty(G, dtype=np.float64)
    s = np.empty(G, dtype=np.float64)
    dp = ctypes.POINTER(ctypes.c_double)
    _check(load().zmc_scan(d.ref, f.ctypes.data_as(dp), s.ctypes.data_as(dp)))
    return f, s


def scan_chunked(spec, chunk_points=0, f=None, sigma=None):
    """(f, sigma) in host memory through the out-of-core entry point: numpy
    float64 arrays (allocated when None), or any host buffers with
    `ctypes`/`data_ptr` (pinned torch tensors take the copies directly)."""
    d = Desc(spec)
    G = validate(spec)
    f = np.empty(G, dtype=np.float64) if f is None else f
    sigma = np.empty(G, dtype=np.float64) if sigma is None else sigma

    def ptr(a):
        return ctypes.c_void_p(a.data_ptr() if hasattr(a, "data_ptr") else a.ctypes.data)

    _check(load().zmc_scan_chunked(d.ref, ptr(f), ptr(sigma), int(chunk_points)))
    return f, sigma


def scan_range(spec, g_begin, g_end, chunk_points=0, f=None, sigma=None):
    """(f, sigma) in host memory for grid points [g_begin, g_end): bitwise the
    same slice of a whole-grid scan (resumable, shardable)."""
    d = Desc(spec)
    n = int(g_end) - int(g_begin)
    f = np.empty(max(n, 0), dtype=np.float64) if f is None else f
    sigma = np.empty(max(n, 0), dtype=np.float64) if sigma is None else sigma

    def ptr(a):
        return ctypes.c_void_p(a.data_ptr() if hasattr(a, "data_ptr") else a.ctypes.data)

    _check(load().zmc_scan_range(d.ref, int(g_begin), int(g_end), ptr(f), ptr(sigma),
                                 int(chunk_points)))
    return f, sigma


def integrate(integrand, domain, parameters, samples, seed=0, precision="fp64", constants=None,
              host=True):
    """One parameter scan, stated as the paper states it (Sec. 2): f(x) is the
    integral of g(y; x) over the box `domain` at every point x of the grid
    spanned by the value lists `parameters`.

    integrand:  a compiled-in family name ("sin_sum", "gauss", "cosexp") or
                the HIP source of `integrand<T>(y, x, p)` (see include/zmc.h)
    domain:     N pairs (lo, hi), one per integration variable
    parameters: M sequences of values (the grid is their outer product)
    constants:  up to 16 values p[] for a source integrand
    host:       True: numpy arrays, streamed through host memory in chunks
                (any grid size); False: float64 device tensors

    Returns (f, sigma), each shaped (len(parameters[0]), ..., len(parameters[M-1]))."""
    from . import workloads
    box = np.asarray(domain, dtype=np.float64).reshape(-1, 2)
    axes = [np.asarray(v, dtype=np.float64).ravel() for v in parameters]
    if integrand in FAMILY and integrand != "user":
        kw = dict(family=integrand)
    else:
        kw = dict(family="user", source=str(integrand),
                  params=np.zeros(0) if constants is None else np.asarray(constants, dtype=np.float64))
    spec = workloads.ScanSpec(axes=axes, lo=box[:, 0], hi=box[:, 1], samples=int(samples),
                              seed=int(seed), precision=precision, name="integrate", **kw)
    shape = spec.shape
    if host:
        f, s = scan_chunked(spec)
    else:
        f, s = scan(spec)
    return f.reshape(shape), s.reshape(shape)


def debug_valu_probe(blocks, iters, stream=None):
    """Launch the VALU calibration load (64 x iters FMAs per lane, blocks x 256
    lanes) on `stream`; returns its float32 output tensor."""
    import torch
    out = torch.empty(int(blocks) * 256, dtype=torch.float32, device="cuda")
    _check(load().zmc_debug_valu_probe(int(blocks), int(iters), ctypes.c_void_p(out.data_ptr()),
                                       _stream_ptr(stream)))
    return out


RATE_OPS = ("xor_b32", "add_f32", "fma_f32", "mad_u64_u32", "bitop3_b32", "exp_f32", "sin_f32",
            "fma_f64")


def debug_rate_probe(op, blocks, iters, stream=None):
    """Launch the instruction-rate load of form `op` (a name of RATE_OPS);
    returns its output tensor (one word per thread)."""
    import torch
    out = torch.empty(blocks * 256, dtype=torch.int64, device="cuda")
    _check(load().zmc_debug_rate_probe(RATE_OPS.index(op), blocks, iters,
                                       ctypes.c_void_p(out.data_ptr()), _stream_ptr(stream)))
    return out


def debug_words(seed, g, w0, count, stream=None):
    """Words w0 .. w0+count-1 of point g's stream from the device generator
    (int64 tensor holding the unsigned values)."""
    import torch
    out = torch.empty(count, dtype=torch.int32, device="cuda")
    _check(load().zmc_debug_words(int(seed) & 0xFFFFFFFFFFFFFFFF, int(g), int(w0), int(count),
                                  ctypes.c_void_p(out.data_ptr()), _stream_ptr(stream)))
    return out.to(torch.int64) & 0xFFFFFFFF


def debug_values(spec, g, s0, count, stream=None):
    """Integrand values of samples s0 .. s0+count-1 at point g, computed on the
    device in the spec's precision (float64 tensor)."""
    import torch
    d_axis = axis_tensor(spec)
    out = torch.empty(count, dtype=torch.float64, device="cuda")
    d = Desc(spec)
    _check(load().zmc_debug_values(d.ref, ctypes.c_void_p(d_axis.data_ptr()), int(g),
                                   int(s0), int(count), ctypes.c_void_p(out.data_ptr()),
                                   _stream_ptr(stream)))
    return out


# ---------------------------------------------------------------- batches ---
def _batch_opts(use_graph=True, parallel_variants=True, pm_groups=0, sm_groups=0,
                pm_min_points=0, cu_count=0, one_kernel=False):
    o = BatchOpts()
    load().zmc_batch_default_opts(ctypes.byref(o))
    o.use_graph = int(bool(use_graph))
    o.parallel_variants = int(bool(parallel_variants))
    o.pm_groups, o.sm_groups, o.pm_min_points = int(pm_groups), int(sm_groups), int(pm_min_points)
    o.cu_count = int(cu_count)
    o.one_kernel = int(bool(one_kernel))
    return o


def _info_dict(info):
    return {k: getattr(info, k) for k, _ in BatchInfo._fields_}


class _DescArray:
    """A contiguous C array of descriptors for a list of ScanSpecs."""

    def __init__(self, specs):
        self.descs = [Desc(sp) for sp in specs]
        self.arr = (ScanDesc * len(specs))(*[d.c for d in self.descs])


def batch_plan(specs, **opts):
    """Host-only plan of a batch: tiles, variants, workspace (dict)."""
    da = _DescArray(specs)
    o = _batch_opts(**opts)
    info = BatchInfo()
    _check(load().zmc_batch_plan(da.arr, len(specs), ctypes.byref(o), ctypes.byref(info)))
    return _info_dict(info)


class Batch:
    """Many scans captured once in a hipGraph; `launch` replays it.

    outputs: list of (f, sigma) float64 device tensors (allocated when None);
    axes: list of device tensors holding each scan's lists (staged by the
    library from the specs when None)."""

    def __init__(self, specs, outputs=None, axes=None, **opts):
        import torch
        self.specs = list(specs)
        n = len(self.specs)
        if outputs is None:
            outputs = []
            for sp in self.specs:
                G = validate(sp)
                outputs.append((torch.empty(G, dtype=torch.float64, device="cuda"),
                                torch.empty(G, dtype=torch.float64, device="cuda")))
        self.outputs = outputs
        self.axes = axes
        self._da = _DescArray(self.specs)
        P = ctypes.c_void_p * n
        self._f = P(*[f.data_ptr() for f, _ in outputs])
        self._s = P(*[s.data_ptr() for _, s in outputs])
        self._a = P(*[a.data_ptr() for a in axes]) if axes is not None else None
        o = _batch_opts(**opts)
        h = ctypes.c_void_p()
        _check(load().zmc_batch_create(self._da.arr, n, self._a, self._f, self._s, ctypes.byref(o),
                                       ctypes.byref(h)))
        self._h = h

    def launch(self, stream=None):
        _check(load().zmc_batch_launch(self._h, _stream_ptr(stream)))

    def info(self):
        info = BatchInfo()
        _check(load().zmc_batch_get_info(self._h, ctypes.byref(info)))
        return _info_dict(info)

    def close(self):
        if getattr(self, "_h", None):
            _check(load().zmc_batch_destroy(self._h))
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def scan_batch(specs, **opts):
    """Run a batch once and return its [(f, sigma)] device tensors."""
    import torch
    b = Batch(specs, **opts)
    b.launch()
    torch.cuda.synchronize()
    out = b.outputs
    b.close()
    return out


def tune_source():
    return load().zmc_tune_source().decode()


# ---------------------------------------------------------------- serving ---
class Server:
    """Continuous-batching request loop (zmc_server_*).  `submit` returns a
    ticket immediately.  Outputs are float64 device tensors that the Server
    keeps alive until they are handed over (`outputs`) or the request is
    released (`release`); `outputs` also releases the request, so a
    long-running caller holds memory only for requests it has not collected.

    Outputs the Server allocates come from a stream of its own on which no
    work is ever queued, so torch's caching allocator never hands it a block
    that pending work on another stream still uses; at hand-over they are
    marked as used on the current stream.  Outputs passed in by the caller
    must not be in use by pending work on other streams when submitted."""

    def __init__(self, hbm_budget_bytes=0, max_slots=0, slice_tiles=0, max_inflight=0, cu_count=0,
                 slice_samples=0, admission="fifo", max_wait_ms=0, slice_us=0):
        o = ServerOpts(int(hbm_budget_bytes), int(max_slots), int(slice_tiles), int(max_inflight),
                       int(cu_count), int(slice_samples), ADMISSION[admission], int(max_wait_ms),
                       int(slice_us))
        h = ctypes.c_void_p()
        _check(load().zmc_server_create(ctypes.byref(o), ctypes.byref(h)))
        self._h = h
        self._keep = {}
        self._alloc_stream = None

    def submit(self, spec, f=None, sigma=None, axis=None):
        import torch
        G = validate(spec)
        if f is None or sigma is None:
            if self._alloc_stream is None:
                self._alloc_stream = torch.cuda.Stream()
            with torch.cuda.stream(self._alloc_stream):
                if f is None:
                    f = torch.empty(G, dtype=torch.float64, device="cuda")
                if sigma is None:
                    sigma = torch.empty(G, dtype=torch.float64, device="cuda")
        d = Desc(spec)
        t = ctypes.c_uint64()
        _check(load().zmc_server_submit(self._h, d.ref,
                                        ctypes.c_void_p(axis.data_ptr()) if axis is not None else None,
                                        ctypes.c_void_p(f.data_ptr()), ctypes.c_void_p(sigma.data_ptr()),
                                        ctypes.byref(t)))
        self._keep[t.value] = (f, sigma, axis)
        return t.value

    def outputs(self, ticket):
        """(f, sigma) of a finished request, handed over to the caller: the
        Server forgets the request (its ticket becomes unknown).  After
        close() every request has finished and its outputs can still be
        collected."""
        import torch
        f, s, _ = self._keep[ticket]
        if getattr(self, "_h", None):
            self.release(ticket)
        else:
            del self._keep[ticket]
        cur = torch.cuda.current_stream()
        f.record_stream(cur)
        s.record_stream(cur)
        return f, s

    def release(self, ticket):
        """Forget a finished request and drop the Server's references to its
        outputs (zmc_server_release; raises while it is still running)."""
        _check(load().zmc_server_release(self._h, int(ticket)))
        self._keep.pop(ticket, None)

    def cancel(self, ticket):
        """Cancels a request that has not been admitted yet (zmc_server_cancel):
        True if it was, False if it has already been admitted or finished."""
        st = load().zmc_server_cancel(self._h, ctypes.c_uint64(int(ticket)))
        if st == 5:
            return False
        _check(st)
        return True

    def poll(self, ticket):
        """(done, status, latency_s)."""
        done = ctypes.c_int32()
        st = ctypes.c_int()
        lat = ctypes.c_double()
        _check(load().zmc_server_poll(self._h, ticket, ctypes.byref(done), ctypes.byref(st),
                                      ctypes.byref(lat)))
        return bool(done.value), st.value, lat.value

    def wait(self, ticket):
        """(status, latency_s) once the request has finished."""
        st = ctypes.c_int()
        lat = ctypes.c_double()
        _check(load().zmc_server_wait(self._h, ticket, ctypes.byref(st), ctypes.byref(lat)))
        return st.value, lat.value

    def stats(self):
        st = ServerStats()
        _check(load().zmc_server_get_stats(self._h, ctypes.byref(st)))
        return {k: getattr(st, k) for k, _ in ServerStats._fields_}

    def close(self):
        """Finish every submitted request and free the server; outputs not yet
        collected stay available through `outputs`."""
        if getattr(self, "_h", None):
            _check(load().zmc_server_destroy(self._h))
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
