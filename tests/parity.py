"""Parity metric between the GPU library and the oracle.

err_f     = |f - f_ref| / max(|f_ref|, sigma_ref * sqrt(n))
err_sigma = |sigma - sigma_ref| / sigma_ref
sigma_ref * sqrt(n) = V sd(g) is the integrand's own scale, so a point whose
integral is near zero is judged against that scale rather than against 0.
Where sigma_ref is 0 (a constant integrand), sigma must be at most
tol_sigma * |f_ref|.

Tolerances: FP64 path 1e-12 on both; FP32-evaluation path 2e-5 on f and
1e-3 on sigma.

Small sample counts (FP32 path only, `small_n=True`): each FP32 sample
carries an absolute rounding error of order 2^-24 times the magnitude of its
intermediates (a SIN_SUM phase of size ~10 over N = 8 terms reaches ~2^-20),
which moves sigma by about that error x V / sqrt(n) however small the sample
spread is.  With n = 2 and two nearly equal samples the spread, and sigma_ref,
can be smaller than that, so for tests of tiny or ragged sample counts the
relative bar is taken against max(sigma_ref, floor) with
    floor = 2^-18 V (1 + |f_ref| / V) / sqrt(n) / tol_sigma.
The full-size workload tests (n >= 4096) use the plain relative bar.
"""
import numpy as np

TOL = {"fp64": (1e-12, 1e-12), "fp32": (2e-5, 1e-3)}


def errors(f, s, f_ref, s_ref, n, precision="fp64", small_n=False, volume=1.0):
    f, s, f_ref, s_ref = (np.asarray(a, dtype=np.float64) for a in (f, s, f_ref, s_ref))
    rn = np.sqrt(float(n))
    scale = np.maximum(np.abs(f_ref), s_ref * rn)
    scale = np.where(scale > 0, scale, 1.0)
    err_f = np.abs(f - f_ref) / scale
    tol_s = TOL[precision][1]
    denom = np.where(s_ref > 0, s_ref, np.abs(f_ref))
    if precision == "fp32" and small_n:
        floor = 2.0 ** -18 * volume * (1.0 + np.abs(f_ref) / volume) / rn / tol_s
        denom = np.maximum(denom, floor)
    with np.errstate(divide="ignore", invalid="ignore"):
        err_s = np.where(denom > 0, np.abs(s - s_ref) / np.where(denom > 0, denom, 1.0),
                         np.where(s == 0.0, 0.0, np.inf))
    # a zero sigma_ref is judged against |f_ref|: sigma <= tol * |f_ref|
    return err_f, err_s


def check(f, s, f_ref, s_ref, n, precision, label="", small_n=False, volume=1.0):
    tf, ts = TOL[precision]
    err_f, err_s = errors(f, s, f_ref, s_ref, n, precision, small_n, volume)
    msg = (f"{label}: max err_f={err_f.max():.3e} (rms {np.sqrt(np.mean(err_f ** 2)):.3e}, tol {tf}) "
           f"max err_sigma={err_s.max():.3e} (rms {np.sqrt(np.mean(err_s ** 2)):.3e}, tol {ts})")
    assert np.all(np.isfinite(f)) and np.all(np.isfinite(s)), label + ": non-finite output"
    assert err_f.max() <= tf and err_s.max() <= ts, msg
    return err_f, err_s, msg
