"""Seeded synthetic scan descriptions (inputs only, no Monte Carlo arithmetic).

This module is shared by the tests, the benchmark and the smoke check: it
builds the parameter lists, boxes, sample counts and seeds of the workloads,
and nothing else.  Both the GPU library binding and the CPU oracle binding
read a `ScanSpec` through its plain attributes.

Workloads (integrands as in the paper's Eq. (2)/(4) for SIN_SUM; GAUSS and
COSEXP are the two further benchmark integrands):
  plain_fp64      1 parameter x1 = linspace(0,1,1000), SIN_SUM, y in [0,1]^4,
                  2^16 samples, seed 42, FP64
  gauss_2p        x1, x2 = linspace(0.1,10,1000) (1e6 points), GAUSS,
                  y in [0,1]^3, 2^14 samples, seed 42
  cosexp_4p       x1..x4 = linspace(-1,1,100) (1e8 points), COSEXP,
                  y in [0,2]x[0,1], 4096 samples, seed 42
  batched_512     512 scans with log-uniform grid sizes in [1e3,1e6], N in
                  2..8, samples in {2^10..2^18}, family uniform, seeds 0..511
  boltzmann_shape 30^3 x 10^3 x 7 = 1.89e8 points, SIN_SUM over the seven
                  parameters, y in [0,1]^5, 1024 samples, seed 5 (out-of-core)
  grid_1e10       10000 x 1000 x 1000 = 1e10 points, SIN_SUM, y in [0,1]^2,
                  16 samples, seed 11 (160 GB of results, streamed in ranges)
"""
from dataclasses import dataclass, field
from typing import List

import numpy as np

FAMILIES = ("sin_sum", "gauss", "cosexp", "const", "linear", "user")
PRECISIONS = ("fp64", "fp32")


@dataclass
class ScanSpec:
    family: str
    axes: List[np.ndarray]
    lo: np.ndarray
    hi: np.ndarray
    samples: int
    seed: int
    precision: str = "fp64"
    name: str = ""
    meta: dict = field(default_factory=dict)
    # family "user": the integrand's source text (a function template
    # integrand<T>(y, x, p), see include/zmc.h) and its constants p
    source: str = ""
    params: np.ndarray = field(default_factory=lambda: np.zeros(0))
    # family "user": FP32 variants with approximate transcendentals
    fast_math: bool = False

    def __post_init__(self):
        self.axes = [np.ascontiguousarray(a, dtype=np.float64).ravel() for a in self.axes]
        self.lo = np.ascontiguousarray(self.lo, dtype=np.float64).ravel()
        self.hi = np.ascontiguousarray(self.hi, dtype=np.float64).ravel()
        self.params = np.ascontiguousarray(self.params, dtype=np.float64).ravel()

    @property
    def M(self):
        return len(self.axes)

    @property
    def N(self):
        return len(self.lo)

    @property
    def G(self):
        g = 1
        for a in self.axes:
            g *= len(a)
        return g

    @property
    def shape(self):
        return tuple(len(a) for a in self.axes)

    def with_(self, **kw):
        d = dict(family=self.family, axes=self.axes, lo=self.lo, hi=self.hi,
                 samples=self.samples, seed=self.seed, precision=self.precision,
                 name=self.name, meta=dict(self.meta), source=self.source, params=self.params,
                 fast_math=self.fast_math)
        d.update(kw)
        return ScanSpec(**d)


def plain_fp64(points=1000, samples=1 << 16, seed=42):
    """Plain FP64 scan: sin(x1 + y1 + y2 + y3 + y4) over [0,1]^4."""
    return ScanSpec("sin_sum", [np.linspace(0.0, 1.0, points)], np.zeros(4), np.ones(4),
                    samples, seed, "fp64", name="plain_fp64_sin_sum_1x1000_N4_n65536")


def gauss_2p(points_per_axis=1000, samples=1 << 14, seed=42, precision="fp32"):
    """Two-parameter grid: exp(-(x1 y1^2 + x2 y2^2 + y3^2)) over [0,1]^3."""
    ax = np.linspace(0.1, 10.0, points_per_axis)
    return ScanSpec("gauss", [ax, ax.copy()], np.zeros(3), np.ones(3), samples, seed,
                    precision, name=f"gauss_2p_{points_per_axis}x{points_per_axis}_N3_n{samples}")


def cosexp_4p(points_per_axis=100, samples=4096, seed=42, precision="fp32"):
    """Four-parameter grid: cos(x1 y1 + x2 y2) exp(-x3^2 y1 y2) + x4 over [0,2]x[0,1]."""
    ax = np.linspace(-1.0, 1.0, points_per_axis)
    return ScanSpec("cosexp", [ax, ax.copy(), ax.copy(), ax.copy()], np.array([0.0, 0.0]),
                    np.array([2.0, 1.0]), samples, seed, precision,
                    name=f"cosexp_4p_{points_per_axis}^4_N2_n{samples}")


def boltzmann_shape(samples=1024, seed=5, precision="fp32"):
    """A grid shaped like the paper's Boltzmann application (Sec. 3.3): three
    momentum components with 30 values, three with 10, and 7 species, i.e.
    1.89e8 points, over a 5-dimensional integral; SIN_SUM over the seven
    parameters stands in for the collision integrand, which the paper does
    not give."""
    axes = [np.linspace(0.0, 1.0, 30)] * 3 + [np.linspace(0.0, 0.5, 10)] * 3 + [np.arange(7.0)]
    return ScanSpec("sin_sum", axes, np.zeros(5), np.ones(5), samples, seed, precision,
                    name=f"boltzmann_shape_30^3x10^3x7_N5_n{samples}")


def grid_1e10(samples=16, seed=11, precision="fp32"):
    """A 10^10-point grid (10000 x 1000 x 1000 parameter values), the upper end
    of the out-of-core scale: 160 GB of f and sigma, more than the device
    holds, streamed to the host in ranges.  SIN_SUM over a 2-dimensional box."""
    axes = [np.linspace(0.0, 1.0, 10000), np.linspace(0.0, 1.0, 1000), np.linspace(0.0, 1.0, 1000)]
    return ScanSpec("sin_sum", axes, np.zeros(2), np.ones(2), samples, seed, precision,
                    name=f"grid_10000x1000x1000_N2_n{samples}")


def cosexp_subsample(G=10**8, k=10**4, seed=42):
    """Sorted flat indices of the sampled points checked on the 1e8-point grid."""
    return np.sort(np.random.default_rng(seed).choice(G, k, replace=False)).astype(np.uint64)


def family_shape(family, N, L, samples, seed, precision="fp32"):
    """One scan of a family at integration dimension N with L values per axis.

    sin_sum keeps one parameter on [0,1]^N; gauss keeps two parameters in
    [0.1,10] (the further dimensions weigh 1); cosexp keeps four parameters in
    [-1,1] on [0,2]x[0,1]^(N-1) (the further dimensions enter the cosine).
    """
    if family == "sin_sum":
        axes = [np.linspace(0.0, 1.0, L)]
        lo, hi = np.zeros(N), np.ones(N)
    elif family == "gauss":
        axes = [np.linspace(0.1, 10.0, L) for _ in range(2)]
        lo, hi = np.zeros(N), np.ones(N)
    elif family == "cosexp":
        axes = [np.linspace(-1.0, 1.0, L) for _ in range(4)]
        lo = np.zeros(N)
        hi = np.ones(N)
        hi[0] = 2.0
    else:
        raise ValueError(family)
    return ScanSpec(family, axes, lo, hi, samples, seed, precision,
                    name=f"{family}_N{N}_L{L}_n{samples}_s{seed}")


_FAMILY_M = {"sin_sum": 1, "gauss": 2, "cosexp": 4}


def batched_512(count=512, seed=3, precision="fp32", dims=(2, 8)):
    """The 512-scan batch: family uniform over the three, N uniform in 2..8,
    grid size log-uniform in [1e3, 1e6] (L = max(2, round(G^(1/M))) values per
    axis), samples uniform over {2^10, ..., 2^18}, Philox seeds 0..count-1.
    `dims` = (smallest, largest) N."""
    rng = np.random.default_rng(seed)
    fams = ["sin_sum", "gauss", "cosexp"]
    out = []
    for i in range(count):
        fam = fams[int(rng.integers(0, 3))]
        N = int(rng.integers(dims[0], dims[1] + 1))
        g_target = float(np.exp(rng.uniform(np.log(1e3), np.log(1e6))))
        M = _FAMILY_M[fam]
        L = max(2, int(round(g_target ** (1.0 / M))))
        samples = 1 << int(rng.integers(10, 19))
        out.append(family_shape(fam, N, L, samples, i, precision))
    return out


def batched_wide(count=96, seed=4, precision="fp32"):
    """Scans shaped like the 512-scan batch with N uniform in 9..16 (the
    integration dimensions above the any-family kernel's), for tuning and
    testing those kernels."""
    return batched_512(count=count, seed=seed, precision=precision, dims=(9, 16))
