"""ctypes binding of the plain-C FP64 oracle (oracle/zmc_oracle.c).

TEST INFRASTRUCTURE ONLY: used by the tests, the smoke check and the
benchmark's CPU-baseline leg; never by the product path.

A scan is described by any object with the attributes
    family   one of "sin_sum", "gauss", "cosexp", "const", "linear", "user"
    axes     sequence of M one-dimensional float64 arrays (parameter lists)
    lo, hi   length-N float64 arrays (the integration box)
    samples  samples per grid point
    seed     Philox key (64 bits)
    source, params   (family "user") the integrand's source text, which
             defines template <typename T> T integrand(const T* y, const T* x,
             const T* p) with __device__ in front, and its constants p
A user integrand is evaluated by compiling that same text as host C++ with
g++ (ISO mode, no FMA contraction; <cmath> functions in double), so the GPU
library and the oracle share the user's text and nothing else.
This module imports nothing from the GPU package.
"""
import ctypes
import hashlib
import os
import subprocess
import tempfile

import numpy as np

from . import build as _build

_FAMILY = {"sin_sum": 0, "gauss": 1, "cosexp": 2, "const": 3, "linear": 4, "user": 5}
_USER_FN = ctypes.CFUNCTYPE(ctypes.c_double, ctypes.POINTER(ctypes.c_double),
                            ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double))


class _Spec(ctypes.Structure):
    _fields_ = [
        ("M", ctypes.c_int32),
        ("N", ctypes.c_int32),
        ("axis_len", ctypes.POINTER(ctypes.c_int64)),
        ("axis_vals", ctypes.POINTER(ctypes.c_double)),
        ("lo", ctypes.POINTER(ctypes.c_double)),
        ("hi", ctypes.POINTER(ctypes.c_double)),
        ("family", ctypes.c_int32),
        ("samples", ctypes.c_uint64),
        ("seed", ctypes.c_uint64),
        ("user", _USER_FN),
        ("params", ctypes.POINTER(ctypes.c_double)),
        ("n_params", ctypes.c_int32),
    ]


_lib = None
_user_libs = {}
_user_dir = None

_USER_SHIM = """// host build of a user integrand for the oracle
#include <cmath>
using namespace std;
#define __device__
#define __host__
%s
extern "C" double zmc_oracle_user(const double* y, const double* x, const double* p) {
  return integrand<double>(y, x, p);
}
"""


def user_function(source):
    """The FP64 host function of a user integrand's source (compiled with g++
    once per source text and process)."""
    global _user_dir
    key = hashlib.sha256(source.encode()).hexdigest()[:16]
    if key not in _user_libs:
        if _user_dir is None:
            _user_dir = tempfile.mkdtemp(prefix="zmc_oracle_user_")
        src = os.path.join(_user_dir, f"user_{key}.cpp")
        lib = os.path.join(_user_dir, f"user_{key}.so")
        with open(src, "w") as fh:
            fh.write(_USER_SHIM % source)
        r = subprocess.run(["g++", "-std=c++17", "-O2", "-ffp-contract=off", "-fPIC", "-shared",
                            src, "-o", lib], capture_output=True, text=True)
        if r.returncode != 0:
            raise ValueError(f"user integrand does not compile for the oracle:\n{r.stderr}")
        dll = ctypes.CDLL(lib)
        fn = _USER_FN(("zmc_oracle_user", dll))
        _user_libs[key] = (dll, fn)
    return _user_libs[key][1]


def load(path=None):
    """Load (building if absent) the oracle library; returns the CDLL."""
    global _lib
    if path is not None:
        return _declare(ctypes.CDLL(path))
    if _lib is None:
        if not os.path.exists(_build.LIB):
            _build.build()
        _lib = _declare(ctypes.CDLL(_build.LIB))
    return _lib


def _declare(lib):
    u32p = ctypes.POINTER(ctypes.c_uint32)
    dp = ctypes.POINTER(ctypes.c_double)
    lib.zmc_oracle_philox4x32_10.argtypes = [u32p, u32p, u32p]
    lib.zmc_oracle_philox4x32_10.restype = None
    lib.zmc_oracle_word.argtypes = [ctypes.c_uint64, ctypes.c_uint64, ctypes.c_uint64]
    lib.zmc_oracle_word.restype = ctypes.c_uint32
    lib.zmc_oracle_grid_size.argtypes = [ctypes.POINTER(_Spec)]
    lib.zmc_oracle_grid_size.restype = ctypes.c_uint64
    lib.zmc_oracle_values.argtypes = [ctypes.POINTER(_Spec), ctypes.c_uint64,
                                      ctypes.c_uint64, ctypes.c_int64, dp]
    lib.zmc_oracle_values.restype = ctypes.c_int
    lib.zmc_oracle_moments.argtypes = [ctypes.POINTER(_Spec), ctypes.c_uint64, dp, dp]
    lib.zmc_oracle_moments.restype = ctypes.c_int
    lib.zmc_oracle_scan.argtypes = [ctypes.POINTER(_Spec), ctypes.POINTER(ctypes.c_uint64),
                                    ctypes.c_int64, dp, dp]
    lib.zmc_oracle_scan.restype = ctypes.c_int
    return lib


class _Marshalled:
    """Keeps the numpy buffers alive while the C struct points into them."""

    def __init__(self, spec):
        axes = [np.ascontiguousarray(a, dtype=np.float64).ravel() for a in spec.axes]
        self.axis_len = np.array([len(a) for a in axes], dtype=np.int64)
        self.axis_vals = (np.concatenate(axes) if axes else np.zeros(1)).astype(np.float64)
        self.lo = np.ascontiguousarray(spec.lo, dtype=np.float64)
        self.hi = np.ascontiguousarray(spec.hi, dtype=np.float64)
        self.params = np.ascontiguousarray(getattr(spec, "params", np.zeros(0)), dtype=np.float64)
        user = user_function(spec.source) if spec.family == "user" else _USER_FN()
        self.struct = _Spec(
            M=len(axes),
            N=len(self.lo),
            axis_len=self.axis_len.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
            axis_vals=self.axis_vals.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
            lo=self.lo.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
            hi=self.hi.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
            family=_FAMILY.get(spec.family, -1),
            samples=int(spec.samples),
            seed=int(spec.seed) & 0xFFFFFFFFFFFFFFFF,
            user=user,
            params=self.params.ctypes.data_as(ctypes.POINTER(ctypes.c_double)) if self.params.size else None,
            n_params=int(self.params.size),
        )


def _check(rc, what):
    if rc != 0:
        raise ValueError(f"oracle {what} failed with code {rc}")


def philox(ctr, key):
    """Philox4x32-10 block: four uint32 words from a 4-word counter and 2-word key."""
    c = (ctypes.c_uint32 * 4)(*[int(v) & 0xFFFFFFFF for v in ctr])
    k = (ctypes.c_uint32 * 2)(*[int(v) & 0xFFFFFFFF for v in key])
    o = (ctypes.c_uint32 * 4)()
    load().zmc_oracle_philox4x32_10(c, k, o)
    return [int(v) for v in o]


def word(seed, g, w):
    """Word w of the stream of grid point g."""
    return int(load().zmc_oracle_word(int(seed) & (2**64 - 1), int(g), int(w)))


def grid_size(spec):
    m = _Marshalled(spec)  # owns the arrays the struct points into
    return int(load().zmc_oracle_grid_size(ctypes.byref(m.struct)))


def values(spec, g, s0=0, count=None):
    """Integrand values of samples s0 .. s0+count-1 at grid point g (float64)."""
    if count is None:
        count = int(spec.samples) - s0
    m = _Marshalled(spec)
    out = np.empty(count, dtype=np.float64)
    _check(load().zmc_oracle_values(ctypes.byref(m.struct), int(g), int(s0), int(count),
                                    out.ctypes.data_as(ctypes.POINTER(ctypes.c_double))),
           "values")
    return out


def moments(spec, g):
    """(mean, M2) of the integrand samples at grid point g."""
    m = _Marshalled(spec)
    mean = ctypes.c_double()
    m2 = ctypes.c_double()
    _check(load().zmc_oracle_moments(ctypes.byref(m.struct), int(g), ctypes.byref(mean),
                                     ctypes.byref(m2)), "moments")
    return mean.value, m2.value


def scan(spec, idx=None):
    """(f, sigma) float64 arrays at the flat grid indices idx (all points if None)."""
    m = _Marshalled(spec)
    if idx is None:
        n = int(load().zmc_oracle_grid_size(ctypes.byref(m.struct)))
        ip = None
    else:
        idx = np.ascontiguousarray(idx, dtype=np.uint64)
        n = len(idx)
        ip = idx.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64))
    f = np.empty(n, dtype=np.float64)
    s = np.empty(n, dtype=np.float64)
    _check(load().zmc_oracle_scan(ctypes.byref(m.struct), ip, n,
                                  f.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                  s.ctypes.data_as(ctypes.POINTER(ctypes.c_double))),
           "scan")
    return f, s
