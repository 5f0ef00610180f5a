"""Exact integrals and variances of the integrand families, derived by hand.

Used by the tests to pin the oracle (and, through it, the GPU path).  These
formulas are independent of the oracle's code: they are the integrals
themselves, written from calculus, plus Gauss-Legendre quadrature from numpy
for the family with no closed form.

SIN_SUM (paper Eq. (2)/(4)): with phi = sum x + sum y over a box with edges
a_k < b_k, h_k = b_k - a_k,
    int e^{i y} dy over [a,b] = e^{i (a+b)/2} 2 sin(h/2),
so  f = prod_k 2 sin(h_k/2) * sin(sum x + sum_k (a_k+b_k)/2)
and E[g^2] = 1/2 - 1/2 prod_k (sin h_k / h_k) cos(2 sum x + sum_k (a_k+b_k)).
GAUSS: the integral factorises, with
    int_a^b e^{-c y^2} dy = sqrt(pi/c)/2 (erf(sqrt(c) b) - erf(sqrt(c) a)),
    c = x_k for k <= M and 1 beyond; E[g^2] takes 2c.
LINEAR: f = V sum (a_k+b_k)/2, Var g = sum h_k^2 / 12.
"""
import numpy as np
from scipy.special import erf
from scipy.stats import binom


def grid_points(spec):
    """(G, M) array of parameter vectors in C order (last axis fastest)."""
    if spec.M == 0:
        return np.zeros((1, 0))
    mesh = np.meshgrid(*spec.axes, indexing="ij")
    return np.stack([m.ravel() for m in mesh], axis=1)


def volume(spec):
    return float(np.prod(spec.hi - spec.lo))


def sin_sum_exact(spec, X=None):
    """(f, Var g) at every grid point for sin(sum x + sum y)."""
    X = grid_points(spec) if X is None else X
    h = spec.hi - spec.lo
    mid = np.sum(spec.lo + spec.hi)
    sx = X.sum(axis=1)
    f = np.prod(2.0 * np.sin(h / 2.0)) * np.sin(sx + mid / 2.0)
    eg2 = 0.5 - 0.5 * np.prod(np.sin(h) / h) * np.cos(2.0 * sx + mid)
    V = volume(spec)
    return f, eg2 - (f / V) ** 2


def _gauss_1d(c, a, b):
    """int_a^b exp(-c y^2) dy for c >= 0 (vectorised over c)."""
    c = np.asarray(c, dtype=np.float64)
    assert np.all(c >= 0.0)
    out = np.empty_like(c)
    small = c < 1e-6
    cs = c[small]
    # Taylor series in c near 0
    out[small] = (b - a) - cs * (b ** 3 - a ** 3) / 3.0 + cs ** 2 * (b ** 5 - a ** 5) / 10.0
    r = np.sqrt(c[~small])
    out[~small] = 0.5 * np.sqrt(np.pi) * (erf(r * b) - erf(r * a)) / r
    return out


def gauss_exact(spec, X=None):
    """(f, Var g) for exp(-(sum_{k<=M} x_k y_k^2 + sum_{k>M} y_k^2)), x_k >= 0,
    over any box: the integral factorises into one-dimensional Gaussian
    integrals, sqrt(pi/c)/2 (erf(sqrt(c) b) - erf(sqrt(c) a))."""
    X = grid_points(spec) if X is None else X
    M, N = spec.M, spec.N
    V = volume(spec)
    f = np.ones(len(X))
    eg2 = np.ones(len(X))
    for k in range(N):
        c = X[:, k] if k < M else np.ones(len(X))
        f *= _gauss_1d(c, spec.lo[k], spec.hi[k])
        eg2 *= _gauss_1d(2.0 * c, spec.lo[k], spec.hi[k])
    eg2 = eg2 / V
    return f, eg2 - (f / V) ** 2


def linear_exact(spec):
    V = volume(spec)
    f = V * np.sum((spec.lo + spec.hi) / 2.0)
    var = np.sum((spec.hi - spec.lo) ** 2) / 12.0
    return np.full(spec.G, f), np.full(spec.G, var)


def gl_nodes(q, a, b):
    x, w = np.polynomial.legendre.leggauss(q)
    return 0.5 * (b - a) * x + 0.5 * (a + b), 0.5 * (b - a) * w


def cosexp_quadrature(spec, X=None, q=64):
    """(f, Var g) for cos(x1 y1 + x2 y2 + sum_{k>=3} y_k) exp(-x3^2 y1 y2) + x4
    by q x q tensor Gauss-Legendre in (y1, y2); the further dimensions are
    integrated exactly: over a box [a_k, b_k] they turn the cosine term into
    prod 2 sin(h_k/2)/h_k times cos(phase + sum (a_k+b_k)/2) (mean over y),
    and the square into 1/2 + 1/2 prod (sin h_k / h_k) cos(2 phase + sum(a_k+b_k))."""
    X = grid_points(spec) if X is None else X
    y1, w1 = gl_nodes(q, spec.lo[0], spec.hi[0])
    y2, w2 = gl_nodes(q, spec.lo[1], spec.hi[1])
    Y1, Y2 = np.meshgrid(y1, y2, indexing="ij")
    W = np.outer(w1, w2)
    h_rest = spec.hi[2:] - spec.lo[2:]
    mid_rest = np.sum(spec.lo[2:] + spec.hi[2:])
    A1 = np.prod(2.0 * np.sin(h_rest / 2.0) / h_rest) if len(h_rest) else 1.0
    A2 = np.prod(np.sin(h_rest) / h_rest) if len(h_rest) else 1.0
    V2 = (spec.hi[0] - spec.lo[0]) * (spec.hi[1] - spec.lo[1])
    Vr = float(np.prod(h_rest)) if len(h_rest) else 1.0
    f = np.empty(len(X))
    var = np.empty(len(X))
    for i, (x1, x2, x3, x4) in enumerate(X):
        ph = x1 * Y1 + x2 * Y2
        e = np.exp(-(x3 * x3) * Y1 * Y2)
        c_mean = A1 * np.cos(ph + mid_rest / 2.0)       # mean of cos over extra dims
        c2_mean = 0.5 + 0.5 * A2 * np.cos(2.0 * ph + mid_rest)
        m1 = np.sum(W * (c_mean * e)) / V2 + x4                       # E[g]
        m2 = np.sum(W * (c2_mean * e * e + 2.0 * x4 * c_mean * e)) / V2 + x4 * x4
        f[i] = V2 * Vr * m1
        var[i] = m2 - m1 * m1
    return f, var


def exact(spec, X=None):
    if spec.family == "sin_sum":
        return sin_sum_exact(spec, X)
    if spec.family == "gauss":
        return gauss_exact(spec, X)
    if spec.family == "cosexp":
        return cosexp_quadrature(spec, X)
    if spec.family == "linear":
        return linear_exact(spec)
    raise ValueError(spec.family)


def coverage_ok(z, label=""):
    """Normal-score checks of a vector of independent z = (f - f_true)/sigma.

    A correct estimator puts 0.27% of points beyond 3 sigma; the count may
    reach the Binomial(G, 0.0027) quantile at 1 - 1e-6.  The mean and the
    variance of z must also be those of a standard normal within 5 standard
    errors."""
    z = np.asarray(z)
    G = len(z)
    out3 = int(np.sum(np.abs(z) > 3.0))
    limit = int(binom.ppf(1.0 - 1e-6, G, 0.0027))
    ok = (out3 <= limit and abs(z.mean()) < 5.0 / np.sqrt(G)
          and abs(z.var() - 1.0) < 5.0 * np.sqrt(2.0 / G) + 5.0 / G)
    msg = (f"{label}: G={G} beyond-3sigma={out3} (limit {limit}) "
           f"mean z={z.mean():.4f} var z={z.var():.4f} within-3sigma={1 - out3 / G:.4%}")
    return ok, msg
