"""Replays of the paper's own test workloads on one MI355X.

* Sec. 3.1, Eq. (2) and Table 1: sin(sum_j y_j + sum_l x_l) over [0,10]^N,
  every x_l in {0, ..., 99} (100^M grid points), 10^4 samples per point,
  M, N in 1..4; the mean relative error dr of Eq. (3) (read with |f_th|) and
  the HToD / DToH / total times the paper reports for one V100.
* Sec. 3.2, Eq. (4) and Table 2: the same integrand over [0,1]^6 with M = 4,
  N = 6, 10^5 samples; the paper splits the 10^8 points into 100 batches of
  10^6 and times one batch per GPU.  One batch here is x1 fixed, x2..x4 over
  all values; the whole grid is also run as one scan on the one GPU.
* Eq. (5) / Fig. 3: the map dr(x1, x2) = mean over x3, x4 of
  |f_th - f| / |f_th| on the whole Eq. (4) grid.

Every scan goes through the C ABI (zmc.py); the theoretical values come from
the closed form below.  Run on the GPU:

    python -m paper_1910_01965_amd.replay [--table1] [--table2] [--fig3]
"""
import argparse
import json
import sys
import time

import numpy as np

from . import workloads as wl

# The paper's printed numbers (one V100 for Table 1; per-batch figures of
# Table 2), reported beside ours as context.
PAPER_TABLE1 = {  # (M, N): (dr, HToD ms, DToH s, total s)
    (1, 1): (0.02512, 0.72227, 0.00010, 0.59343), (1, 2): (0.25034, 0.84085, 0.00011, 0.57227),
    (1, 3): (1.19949, 0.70653, 0.00010, 0.59330), (1, 4): (6.19901, 0.96030, 0.00010, 0.60408),
    (2, 1): (0.03379, 1.14849, 0.00012, 0.61858), (2, 2): (0.16417, 1.01440, 0.00013, 0.59581),
    (2, 3): (0.87280, 1.19109, 0.00012, 0.61055), (2, 4): (4.12216, 1.13764, 0.00013, 0.62169),
    (3, 1): (0.02927, 1.23856, 0.00200, 1.26269), (3, 2): (0.15052, 1.19336, 0.00303, 1.51221),
    (3, 3): (0.78052, 1.37538, 0.00197, 1.78097), (3, 4): (4.05029, 1.41807, 0.00268, 2.07094),
    (4, 1): (0.08806, 2.79922, 0.60880, 64.8745), (4, 2): (0.55222, 2.68347, 0.61748, 91.5998),
    (4, 3): (3.55857, 2.77383, 0.59681, 118.275), (4, 4): (22.62904, 2.64370, 0.59422, 147.347),
}
PAPER_TABLE2_V100_BATCH_S = 18.19497   # GPU evaluation time per 10^6-point batch
PAPER_TABLE2_TOTAL_S = 721.20234       # all 100 batches on the 3-node, 7-GPU cluster


def sin_sum_exact(sum_x, lo, hi):
    """Integral of sin(c + sum_k y_k) over the box prod_k [lo_k, hi_k] for
    every c in sum_x: the imaginary part of e^{ic} prod_k (e^{i hi_k} -
    e^{i lo_k}) / i."""
    w = np.prod((np.exp(1j * np.asarray(hi, float)) - np.exp(1j * np.asarray(lo, float))) / 1j)
    return np.imag(np.exp(1j * np.asarray(sum_x, float)) * w)


def sin_sum_spread(sum_x, lo, hi):
    """V times the standard deviation of sin(c + sum_k y_k) for y uniform on
    the box (volume V): E[sin^2] = (1 - E[cos 2(c + sum y)]) / 2 with
    E[e^{2i(c + sum y)}] = e^{2ic} prod_k (e^{2i hi_k} - e^{2i lo_k}) / (2i h_k)."""
    lo, hi = np.asarray(lo, float), np.asarray(hi, float)
    h = hi - lo
    V = float(np.prod(h))
    w2 = np.prod((np.exp(2j * hi) - np.exp(2j * lo)) / (2j * h))
    e_sq = 0.5 * (1.0 - np.real(np.exp(2j * np.asarray(sum_x, float)) * w2))
    mean = sin_sum_exact(sum_x, lo, hi) / V
    return V * np.sqrt(np.maximum(e_sq - mean ** 2, 0.0))


def grid_sum(spec):
    """sum_l x_l at every grid point of `spec` (C order, last axis fastest)."""
    s = np.zeros(1)
    for a in spec.axes:
        s = (s[:, None] + a[None, :]).ravel()
    return s


def delta_r(f, f_th):
    """Eq. (3) with |f_th| in the denominator."""
    return float(np.mean(np.abs(f_th - f) / np.abs(f_th)))


def eq2_spec(M, N, samples, precision, seed=42):
    return wl.ScanSpec("sin_sum", [np.arange(100.0)] * M, np.zeros(N), np.full(N, 10.0), samples,
                       seed, precision, name=f"eq2_M{M}_N{N}_n{samples}")


def eq4_spec(samples, precision, x1=None, seed=42):
    """Eq. (4): M = 4, N = 6 over [0,1]^6; x1 = one value gives one of the
    paper's 10^6-point batches."""
    axes = [np.arange(100.0)] * 4
    if x1 is not None:
        axes = [np.array([float(x1)])] + axes[1:]
    return wl.ScanSpec("sin_sum", axes, np.zeros(6), np.ones(6), samples, seed, precision,
                       name=f"eq4_{'batch' if x1 is not None else 'grid'}_n{samples}")


def timed_scan(spec):
    """One scan with the paper's three phases timed: HToD (parameter lists to
    the device), evaluation (the library's kernels, device time), DToH (f and
    sigma back to host memory); plus the main kernel's own duration."""
    import torch
    from . import zmc
    G = zmc.validate(spec)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    d_axis = zmc.axis_tensor(spec)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    f = torch.empty(G, dtype=torch.float64, device="cuda")
    s = torch.empty(G, dtype=torch.float64, device="cuda")
    stream = torch.cuda.current_stream()
    ev = (torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
    for e in ev:  # creates the underlying HIP events
        e.record(stream)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    zmc.scan_device(spec, d_axis, f, s, stream=stream, events=(ev[0].cuda_event, ev[1].cuda_event))
    torch.cuda.synchronize()
    t3 = time.perf_counter()
    fh, sh = f.cpu().numpy(), s.cpu().numpy()
    t4 = time.perf_counter()
    return fh, sh, {"htod_ms": (t1 - t0) * 1e3, "eval_s": t3 - t2, "kernel_s": ev[0].elapsed_time(ev[1]) / 1e3,
                    "dtoh_s": t4 - t3, "total_s": (t1 - t0) + (t3 - t2) + (t4 - t3),
                    "samples_per_s": G * spec.samples / (t3 - t2)}


def table1(samples=10_000, precision="fp64", Ms=(1, 2, 3, 4), Ns=(1, 2, 3, 4), log=None):
    rows = []
    for M in Ms:
        for N in Ns:
            spec = eq2_spec(M, N, samples, precision)
            timed_scan(eq2_spec(M, N, 64, precision))  # warm the kernel variant
            f, _, t = timed_scan(spec)
            dr = delta_r(f, sin_sum_exact(grid_sum(spec), spec.lo, spec.hi))
            p = PAPER_TABLE1[(M, N)]
            row = {"M": M, "N": N, "samples": samples, "precision": precision, "dr": dr, **t,
                   "paper_dr": p[0], "paper_htod_ms": p[1], "paper_dtoh_s": p[2], "paper_total_s": p[3]}
            rows.append(row)
            if log:
                log(f"table1 M={M} N={N} n={samples} {precision}: dr {dr:.5f} (paper {p[0]}), "
                    f"total {t['total_s']:.4f} s (paper {p[3]} s)")
    return rows


def table2_batch(samples=100_000, precision="fp64", x1=0, log=None):
    spec = eq4_spec(samples, precision, x1=x1)
    timed_scan(eq4_spec(64, precision, x1=x1))
    f, _, t = timed_scan(spec)
    dr = delta_r(f, sin_sum_exact(grid_sum(spec), spec.lo, spec.hi))
    out = {"points": spec.G, "samples": samples, "precision": precision, "dr": dr, **t,
           "paper_v100_batch_s": PAPER_TABLE2_V100_BATCH_S,
           "speedup_vs_v100_batch": PAPER_TABLE2_V100_BATCH_S / t["eval_s"]}
    if log:
        log(f"table2 batch x1={x1} {precision}: eval {t['eval_s']:.4f} s (paper V100 "
            f"{PAPER_TABLE2_V100_BATCH_S} s per batch), dr {dr:.5f}")
    return out


def dr_map(f, spec, signed=False):
    """Eq. (5): dr(x1, x2) over the (x1, x2) values of an Eq. (4) grid, the
    mean over x3, x4 of |f_th - f| / |f_th| (signed=True: divided by f_th
    itself, as Eq. (5) is printed)."""
    f_th = sin_sum_exact(grid_sum(spec), spec.lo, spec.hi)
    L = [len(a) for a in spec.axes]
    den = f_th if signed else np.abs(f_th)
    return (np.abs(f_th - f) / den).reshape(L[0], L[1], L[2] * L[3]).mean(axis=2)


def expected_dr_map(spec):
    """The map crude Monte Carlo gives in expectation: |f - f_th| has mean
    sqrt(2/pi) V sd(g) / sqrt(n) at every point."""
    sx = grid_sum(spec)
    e = np.sqrt(2.0 / np.pi) * sin_sum_spread(sx, spec.lo, spec.hi) / np.sqrt(spec.samples)
    r = e / np.abs(sin_sum_exact(sx, spec.lo, spec.hi))
    L = [len(a) for a in spec.axes]
    return r.reshape(L[0], L[1], L[2] * L[3]).mean(axis=2)


def fig3(samples=100_000, precision="fp64", log=None):
    spec = eq4_spec(samples, precision)
    timed_scan(eq4_spec(64, precision, x1=0))
    f, _, t = timed_scan(spec)
    m = dr_map(f, spec)
    ms = dr_map(f, spec, signed=True)
    me = expected_dr_map(spec)
    out = {"points": spec.G, "samples": samples, "precision": precision, **t,
           "dr_map_max": float(m.max()), "dr_map_mean": float(m.mean()),
           "dr_map_median": float(np.median(m)), "expected_map_max": float(me.max()),
           "expected_map_median": float(np.median(me)),
           "signed_map_max": float(ms.max()), "signed_map_min": float(ms.min()),
           "paper_total_cluster_s": PAPER_TABLE2_TOTAL_S}
    if log:
        log(f"fig3 whole grid {precision}: eval {t['eval_s']:.3f} s for {spec.G} points "
            f"(paper cluster total {PAPER_TABLE2_TOTAL_S} s); dr(x1,x2) max {m.max():.4f}, "
            f"median {np.median(m):.4f} (crude-MC expectation: max {me.max():.4f}, median "
            f"{np.median(me):.4f}); with signed f_th: {ms.min():.4f} .. {ms.max():.4f}")
    return out, m


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--table1", action="store_true")
    ap.add_argument("--table2", action="store_true")
    ap.add_argument("--fig3", action="store_true")
    ap.add_argument("--precisions", default="fp64,fp32")
    ap.add_argument("--table1-samples", default="10000")
    ap.add_argument("--ms", default="1,2,3,4", help="Table 1 values of M")
    ap.add_argument("--map-out", default=None, help="write the dr(x1,x2) map (CSV)")
    args = ap.parse_args(argv)
    if not (args.table1 or args.table2 or args.fig3):
        args.table1 = args.table2 = args.fig3 = True
    import torch
    if not torch.cuda.is_available():
        raise SystemExit("the replays need a GPU")

    def log(msg):
        print(msg, file=sys.stderr, flush=True)

    report = {}
    precisions = args.precisions.split(",")
    if args.table1:
        Ms = tuple(int(m) for m in args.ms.split(","))
        report["table1"] = [r for p in precisions for n in args.table1_samples.split(",")
                            for r in table1(int(n), p, Ms=Ms, log=log)]
    if args.table2:
        report["table2_batch"] = [table2_batch(precision=p, log=log) for p in precisions]
    if args.fig3:
        report["fig3"] = []
        for p in precisions:
            out, m = fig3(precision=p, log=log)
            report["fig3"].append(out)
            if args.map_out and p == precisions[0]:
                np.savetxt(args.map_out, m, delimiter=",", fmt="%.6g")
    print(json.dumps(report))


if __name__ == "__main__":
    main()
