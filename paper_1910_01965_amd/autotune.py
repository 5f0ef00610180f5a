"""Autotuner for the batched planner's tile shapes (writes tune_table.txt).

For every kernel variant (family, precision, N) the tuner times the batch
path on that variant's scans of the 512-scan batch shape generator (sample
counts capped to keep a sweep short) with candidate point-major tile lengths,
and on small grids it times point-major against sample-major tiles to find
the grid size where point-major starts to win.  The fastest candidate wins;
ties within 1% go to the longer tile (fewer split partials).  Output lines:

    family precision N pm_groups sm_groups pm_min_points

The library reads the table from tune_table.txt next to libzmc.so (or
$ZMC_TUNE_TABLE).  Run on the GPU:  python -m paper_1910_01965_amd.autotune
"""
import argparse
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
DEFAULT_OUT = os.path.join(HERE, "tune_table.txt")
PM_CANDIDATES = (128, 256, 512, 1024, 2048, 4096, 8192)
SM_GROUPS = 16384
PM_MIN_CANDIDATES = (128, 512, 2048, 8192, 32768)


def _time_batch(zmc, specs, reps, **opts):
    import torch
    b = zmc.Batch(specs, **opts)
    b.launch()
    torch.cuda.synchronize()
    best = float("inf")
    for _ in range(reps):
        t0 = time.perf_counter()
        b.launch()
        torch.cuda.synchronize()
        best = min(best, time.perf_counter() - t0)
    b.close()
    return best


def variant_specs(family, precision, N, max_samples):
    from . import workloads as wl
    pool = wl.batched_512(precision=precision) if N <= 8 else wl.batched_wide(precision=precision)
    out = [s for s in pool if s.family == family and s.N == N]
    if not out:
        out = [wl.family_shape(family, N, 64, 1 << 14, 0, precision)]
    return [s.with_(samples=min(s.samples, max_samples)) for s in out]


def tune_pm_groups(zmc, specs, reps, log):
    times = {}
    for c in PM_CANDIDATES:
        times[c] = _time_batch(zmc, specs, reps, pm_groups=c, pm_min_points=1)
    best = min(times.values())
    choice = max(c for c, t in times.items() if t <= best * 1.01)
    log("    pm_groups " + " ".join(f"{c}:{t * 1e3:.2f}ms" for c, t in times.items()) + f" -> {choice}")
    return choice


def tune_pm_min(zmc, family, precision, N, pm_groups, reps, log):
    """Smallest grid at which point-major tiles beat sample-major tiles for
    one scan running alone (2^14 samples): below it a grid's point-major
    tiles are too few to fill the GPU.  Judged alone, the threshold serves
    the latency of small requests (a small grid alone finishes several times
    sooner in sample-major tiles); in a large batch, where point-major tiles
    of every size keep the GPU full, scans below it carry only a small share
    of the samples."""
    from . import workloads as wl
    choice = 2 * PM_MIN_CANDIDATES[-1]
    M = wl.family_shape(family, N, 2, 4, 0, precision).M
    for G in PM_MIN_CANDIDATES:
        L = max(2, int(round(G ** (1.0 / M))))
        sp = wl.family_shape(family, N, L, 1 << 14, 7, precision)
        t_pm = _time_batch(zmc, [sp], reps, pm_groups=pm_groups, pm_min_points=1)
        t_sm = _time_batch(zmc, [sp], reps, pm_groups=pm_groups, pm_min_points=1 << 40,
                           sm_groups=SM_GROUPS)
        log(f"    G={sp.G}: point-major {t_pm * 1e3:.2f} ms, sample-major {t_sm * 1e3:.2f} ms")
        if t_pm <= t_sm:
            choice = sp.G
            break
    return choice


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=DEFAULT_OUT)
    ap.add_argument("--precisions", default="fp32,fp64")
    ap.add_argument("--families", default="sin_sum,gauss,cosexp")
    ap.add_argument("--dims", default="2,3,4,5,6,7,8")
    ap.add_argument("--max-samples", type=int, default=1 << 15)
    ap.add_argument("--reps", type=int, default=2)
    ap.add_argument("--merge", action="store_true",
                    help="keep the rows of the existing table for variants not tuned in this run")
    args = ap.parse_args(argv)

    import torch
    sys.path.insert(0, os.path.dirname(HERE))
    from . import zmc
    if not torch.cuda.is_available():
        raise SystemExit("the autotuner needs a GPU")

    def log(msg):
        print(msg, file=sys.stderr, flush=True)

    rows = []
    for precision in args.precisions.split(","):
        for family in args.families.split(","):
            for N in (int(x) for x in args.dims.split(",")):
                if family == "cosexp" and N < 2:
                    continue
                log(f"tuning {family} {precision} N={N}")
                specs = variant_specs(family, precision, N, args.max_samples)
                pm = tune_pm_groups(zmc, specs, args.reps, log)
                pmin = tune_pm_min(zmc, family, precision, N, pm, args.reps, log)
                rows.append((family, precision, N, pm, SM_GROUPS, pmin))
    if args.merge and os.path.exists(args.out):
        tuned = {(r[0], r[1], r[2]) for r in rows}
        kept = []
        with open(args.out) as fh:
            for line in fh:
                f = line.split("#", 1)[0].split()
                if len(f) == 6 and (f[0], f[1], int(f[2])) not in tuned:
                    kept.append((f[0], f[1], int(f[2]), int(f[3]), int(f[4]), int(f[5])))
        rows = sorted(kept + rows, key=lambda r: (r[1] != "fp32", ("sin_sum", "gauss", "cosexp").index(r[0])
                                                  if r[0] in ("sin_sum", "gauss", "cosexp") else 9, r[2]))
    props = torch.cuda.get_device_properties(0)
    with open(args.out + ".tmp", "w") as fh:
        fh.write("# zmc tile-shape table, written by paper_1910_01965_amd/autotune.py on "
                 f"{torch.cuda.get_device_name(0)} ({getattr(props, 'gcnArchName', '?')}, "
                 f"{props.multi_processor_count} CUs)\n")
        fh.write("# family precision N pm_groups sm_groups pm_min_points\n")
        for r in rows:
            fh.write(" ".join(str(x) for x in r) + "\n")
    os.replace(args.out + ".tmp", args.out)
    log(f"wrote {args.out} ({len(rows)} variants)")


if __name__ == "__main__":
    main()
