"""Python binding of libzmc (include/zmc.h): argument marshalling only.

Every step of the scan runs in the HIP library; this module converts a
`ScanSpec` (see workloads.py) into the C descriptor, hands torch device
buffers and streams to the library, and raises on a non-zero status.  It
fails loudly when libzmc.so has not been built: there is no fallback.
"""
import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libzmc.so")

FAMILY = {"sin_sum": 0, "gauss": 1, "cosexp": 2, "const": 3, "linear": 4}
PRECISION = {"fp64": 0, "fp32": 1}
MODE = {"auto": 0, "point_major": 1, "sample_major": 2}
MODE_NAME = {v: k for k, v in MODE.items()}
STATUS = {0: "ZMC_OK", 1: "ZMC_E_INVALID", 2: "ZMC_E_NOMEM", 3: "ZMC_E_DEVICE",
          4: "ZMC_E_UNSUPPORTED", 5: "ZMC_E_BUSY"}

EXPORTS = ("zmc_last_error", "zmc_version", "zmc_validate", "zmc_plan", "zmc_scan",
           "zmc_scan_device", "zmc_scan_device_ex", "zmc_debug_words", "zmc_debug_values")


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
        lib.zmc_scan_device.argtypes = [descp, vp, vp, vp, vp]
        lib.zmc_scan_device_ex.argtypes = [descp, vp, vp, vp, ctypes.POINTER(LaunchOpts), vp]
        lib.zmc_debug_words.argtypes = [ctypes.c_uint64, ctypes.c_uint64, ctypes.c_uint64,
                                        ctypes.c_int64, vp, vp]
        lib.zmc_debug_values.argtypes = [descp, vp, ctypes.c_uint64, ctypes.c_uint64,
                                         ctypes.c_int64, vp, vp]
        for name in ("zmc_validate", "zmc_plan", "zmc_scan", "zmc_scan_device",
                     "zmc_scan_device_ex", "zmc_debug_words", "zmc_debug_values"):
            getattr(lib, name).restype = ctypes.c_int
        _lib = lib
    return _lib


def _check(status):
    if status != 0:
        raise ZmcError(status, load().zmc_last_error().decode())


class Desc:
    """A C descriptor for one ScanSpec; keeps its host arrays alive."""

    def __init__(self, spec, precision=None):
        self.spec = spec
        self.axis_len = np.array([len(a) for a in spec.axes], dtype=np.int64)
        self.axis_vals = (np.concatenate(spec.axes) if spec.axes else np.zeros(1)).astype(np.float64)
        self.lo = np.ascontiguousarray(spec.lo, dtype=np.float64)
        self.hi = np.ascontiguousarray(spec.hi, dtype=np.float64)
        prec = precision or spec.precision
        self.c = ScanDesc(
            M=len(spec.axes), N=len(self.lo),
            axis_len=self.axis_len.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
            axis_vals=self.axis_vals.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
            lo=self.lo.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
            hi=self.hi.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
            family=FAMILY.get(spec.family, -1), precision=PRECISION.get(prec, -1),
            params=None, n_params=0, samples=int(spec.samples),
            seed=int(spec.seed) & 0xFFFFFFFFFFFFFFFF)

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
    tensors of G elements; d_axis holds the parameter lists on the device.
    `events` = (begin, end) raw hipEvent_t handles recorded around the main
    kernel."""
    o = _opts(mode, block, splits, events=events)
    d = Desc(spec)
    _check(load().zmc_scan_device_ex(d.ref, ctypes.c_void_p(d_axis.data_ptr()),
                                     ctypes.c_void_p(f.data_ptr()), ctypes.c_void_p(sigma.data_ptr()),
                                     ctypes.byref(o) if o else None, _stream_ptr(stream)))


def scan(spec, mode=None, block=None, splits=None, stream=None):
    """(f, sigma) float64 device tensors for every grid point of `spec`."""
    import torch
    G = validate(spec)
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
