"""Parity metric between the GPU library and the oracle.

err_f     = |f - f_ref| / max(|f_ref|, sigma_ref * sqrt(n))
err_sigma = |sigma - sigma_ref| / sigma_ref
sigma_ref * sqrt(n) = V sd(g) is the integrand's own scale, so a point whose
integral is near zero is judged against that scale rather than against 0.
Where sigma_ref is 0 (a constant integrand), sigma must be below
1e-12 * |f_ref| (or 1e-300).

Tolerances: FP64 path 1e-12 on both; FP32-evaluation path 2e-5 on f and
1e-3 on sigma.
"""
import numpy as np

TOL = {"fp64": (1e-12, 1e-12), "fp32": (2e-5, 1e-3)}


def errors(f, s, f_ref, s_ref, n):
    f, s, f_ref, s_ref = (np.asarray(a, dtype=np.float64) for a in (f, s, f_ref, s_ref))
    scale = np.maximum(np.abs(f_ref), s_ref * np.sqrt(float(n)))
    scale = np.where(scale > 0, scale, 1.0)
    err_f = np.abs(f - f_ref) / scale
    with np.errstate(divide="ignore", invalid="ignore"):
        err_s = np.where(s_ref > 0, np.abs(s - s_ref) / np.where(s_ref > 0, s_ref, 1.0),
                         np.where(np.abs(s) <= 1e-12 * np.maximum(np.abs(f_ref), 1e-288), 0.0, np.inf))
    return err_f, err_s


def check(f, s, f_ref, s_ref, n, precision, label=""):
    tf, ts = TOL[precision]
    err_f, err_s = errors(f, s, f_ref, s_ref, n)
    msg = (f"{label}: max err_f={err_f.max():.3e} (rms {np.sqrt(np.mean(err_f ** 2)):.3e}, tol {tf}) "
           f"max err_sigma={err_s.max():.3e} (rms {np.sqrt(np.mean(err_s ** 2)):.3e}, tol {ts})")
    assert np.all(np.isfinite(f)) and np.all(np.isfinite(s)), label + ": non-finite output"
    assert err_f.max() <= tf and err_s.max() <= ts, msg
    return err_f, err_s, msg
