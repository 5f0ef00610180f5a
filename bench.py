"""Throughput benchmark of the MI355X parameter-scan Monte Carlo.

A step is one whole scan of the two-parameter Gaussian grid (1000 x 1000
points, y in [0,1]^3, 2^14 samples per point, Philox seed 42) on one GPU:
planning, point decoding, Philox words, uniform map, integrand, per-lane
Kahan sums, FP64 merges, split merge and the f / sigma writes.  The parameter
lists and the output buffers are resident in HBM before the timed region.

Prints ONE JSON line on stdout.  Beside the headline: the FP64 path on the
same workload; per-step latency percentiles; the roofline of the main kernel
and of the 1e8-point COSEXP scan's kernels (VALU-bound: algorithmic
lane-operations per sample from valu_ops_per_sample against the FP32 vector
peak, plus HBM traffic and the fraction reached by executed VALU instructions
from committed rocprofv3 counter records of the very kernels built); the
512-scan batch and a held-out draw; the serving workload as specified (200
req/s Poisson arrivals for 60 s, seed 7, 64 GiB budget) against the same
trace launched back to back, plus shortest-first admission and a steady load
over short windows; the CPU oracle timed on a bounded sample of the same
workload; and the paper's own throughput figures as context.  The whole run
keeps within --time-budget seconds (the serving window shrinks, and says so,
when it would not).

    python bench.py [--steps K] [--warmup W] [--gpus 1]
    python bench.py --rate-probe | --valu-probe | --copy-probe   (calibration loads)
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "MC samples/s & grid pts/s on 1 MI355X (fp32 vs fp64); p50/p99 scan latency"

# MI355X VALU peak in 32-bit lane-operations: 256 CUs x 128 lanes per clock
# x 2.4 GHz = 7.864e13/s, i.e. the published FP32 vector peak of 157.3 TFLOP/s
# with an FMA counted as one operation (2 FLOP).  On gfx950 the two-operand
# (VOP2) ALU forms issue at that rate; three-operand (VOP3) forms such as
# v_mad_u64_u32 and v_bitop3_b32 at half of it; transcendentals at a quarter.
VALU_PEAK = 256 * 128 * 2.4e9

# Per-dispatch counter readings (HBM bytes, VALU instructions) of the kernels
# the line reports on, taken with rocprofv3 --pmc and keyed by the id of the
# kernel they were taken on (paper_1910_01965_amd/kernel_ids.py): a reading is
# used only while that kernel is the one built, else the figures are null.
RECORDS = os.path.join(ROOT, "profiles", "counter_records.txt")


def counter_records(path=RECORDS):
    """[{kernel_id, kernel, workload, fetch_bytes, write_bytes, valu_insts,
    valu_pairs, summary}] from the committed record file."""
    out = []
    if not os.path.exists(path):
        return out
    with open(path) as fh:
        for line in fh:
            f = line.split("#", 1)[0].split()
            if not f:
                continue
            if len(f) != 8:
                raise ValueError(f"{path}: malformed record: {line.strip()}")
            out.append({"kernel_id": f[0], "kernel": f[1], "workload": f[2],
                        "fetch_bytes": float(f[3]), "write_bytes": float(f[4]),
                        "valu_insts": float(f[5]), "valu_pairs": float(f[6]), "summary": f[7]})
    return out


def counter_record(kernel, workload, built_id, records=None):
    """The record of `kernel` (mangled name) on `workload` taken on the kernel
    now built (id `built_id`), or None."""
    for r in counter_records() if records is None else records:
        if r["kernel"] == kernel and r["workload"] == workload and r["kernel_id"] == built_id:
            return r
    return None


def roofline(kernel, workload, family, N, samples, kernel_ms, ids, label):
    """The roofline block of one kernel: algorithmic lane-operations per
    second (valu_ops_per_sample x samples / kernel time) against VALU_PEAK,
    plus, when a counter record of this very kernel exists, the HBM traffic
    per dispatch and the fraction of the peak that its executed VALU
    instructions (rocprofv3 SQ_INSTS_VALU x 64 lanes) reach."""
    w = valu_ops_per_sample(family, N)
    achieved = w * samples / (kernel_ms / 1e3)
    built = ids.get(kernel)
    rec = counter_record(kernel, workload, built) if built else None
    out = {"bound": "alu", "achieved": achieved / 1e12, "peak": VALU_PEAK / 1e12,
           "unit": "T lane-op/s", "frac": achieved / VALU_PEAK,
           "traffic": rec["fetch_bytes"] + rec["write_bytes"] if rec else None,
           "kernel": label, "kernel_id": built, "kernel_ms": kernel_ms, "ops_per_sample": w,
           "samples_per_launch": samples,
           "ops_basis": "algorithmic: Philox4x32-10 10N (2.5N rounds x 4), uniform map 2N, "
                        "integrand, compensated sums 8, per sample"}
    if rec:
        lane_ops = rec["valu_insts"] * 64.0
        out["valu_counters"] = {
            "valu_insts_per_sample": lane_ops / samples,
            "issue_slots_per_sample": (rec["valu_insts"] - rec["valu_pairs"]) * 64.0 / samples,
            "achieved": lane_ops / (kernel_ms / 1e3) / 1e12, "unit": "T lane-op/s",
            "frac": lane_ops / (kernel_ms / 1e3) / VALU_PEAK,
            "what": "executed VALU lane-instructions (SQ_INSTS_VALU x 64, per dispatch) / live "
                    "kernel time / peak",
            "source": rec["summary"]}
    else:
        out["valu_counters"] = None
    return out


def valu_ops_per_sample(family, N):
    """Algorithmic 32-bit lane-operations per sample: Philox4x32-10 needs N/4
    blocks per sample, i.e. 2.5N rounds x (2 wide multiplies + 2 three-way
    xors); the uniform map N conversions + N FMAs; the integrand (GAUSS: N
    mul + N FMA + 1 exp; SIN_SUM: N adds + 1 sin; COSEXP: 2 FMA + (N-2) adds
    + 1 cos + 2 mul + 1 exp + 1 add); the compensated accumulation 8."""
    rng = 2.5 * N * 4
    mapping = 2 * N
    integrand = {"gauss": 2 * N + 1, "sin_sum": N + 1, "cosexp": N + 5}.get(family, N)
    return float(rng + mapping + integrand + 8)


def mix_roofline(specs, seconds):
    """Roofline of a whole mix of scans (a batch, a served trace): every scan's
    algorithmic lane-operations (valu_ops_per_sample x samples) over the wall
    time of the mix, against VALU_PEAK."""
    ops = sum(sp.G * sp.samples * valu_ops_per_sample(sp.family, sp.N) for sp in specs)
    samples = sum(sp.G * sp.samples for sp in specs)
    achieved = ops / seconds
    return {"bound": "alu", "achieved": achieved / 1e12, "peak": VALU_PEAK / 1e12,
            "unit": "T lane-op/s", "frac": achieved / VALU_PEAK,
            "ops_per_sample_mean": ops / samples,
            "what": "algorithmic lane-operations of every scan in the mix / its wall time"}


def grid_1e10_run():
    """The 10^10-point grid (160 GB of f and sigma) streamed to the host as
    twenty ranges of 5e8 points through two reused pinned 4 GB arrays, as a
    caller without 160 GB of host memory runs it: seconds for the whole grid
    and the rate at which results reach host memory."""
    import torch
    from paper_1910_01965_amd import workloads as wl
    from paper_1910_01965_amd import zmc
    spec = wl.grid_1e10()
    step = 500_000_000
    fp = torch.empty(step, dtype=torch.float64, pin_memory=True)
    sp = torch.empty(step, dtype=torch.float64, pin_memory=True)
    ranges = []
    t0 = time.perf_counter()
    for g0 in range(0, spec.G, step):
        g1 = min(spec.G, g0 + step)
        t1 = time.perf_counter()
        zmc.scan_range(spec, g0, g1, 0, fp[: g1 - g0], sp[: g1 - g0])
        ranges.append(time.perf_counter() - t1)
        log(f"grid 1e10: range [{g0}, {g1}) {ranges[-1]:.3f} s")
    total = time.perf_counter() - t0
    finite = bool(torch.isfinite(fp).all()) and bool(torch.isfinite(sp).all())
    del fp, sp
    return {"workload": spec.name, "grid_points": spec.G, "samples_per_point": spec.samples,
            "result_bytes": 16 * spec.G, "ranges": len(ranges), "range_points": step,
            "seconds": total, "pts_per_s": spec.G / total,
            "host_gb_per_s": 16 * spec.G / total / 1e9,
            "range_seconds_min_max": [min(ranges), max(ranges)], "last_range_finite": finite}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def time_path(spec, steps, warmup, events=True):
    """`steps` back-to-back scans of `spec` on the current stream, bracketed by
    synchronisations: wall time, and with `events` the device time of every
    main kernel and of every step (timing events recorded around each scan;
    on the shortest scans they add a few percent to the wall time)."""
    import torch
    from paper_1910_01965_amd import zmc
    G = zmc.validate(spec)
    d_axis = zmc.axis_tensor(spec)
    f = torch.empty(G, dtype=torch.float64, device="cuda")
    s = torch.empty(G, dtype=torch.float64, device="cuda")
    stream = torch.cuda.current_stream()
    for _ in range(warmup):
        zmc.scan_device(spec, d_axis, f, s, stream=stream)
    if not events:
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for i in range(steps):
            zmc.scan_device(spec, d_axis, f, s, stream=stream)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        ok = bool(torch.isfinite(f).all()) and bool(torch.isfinite(s).all())
        return dict(wall_s=wall, finite=ok, plan=zmc.plan(spec))
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(steps)]
    step_ev = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
    for a, b in ev:  # create the underlying HIP events
        a.record(stream)
        b.record(stream)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    step_ev[0].record(stream)
    for i in range(steps):
        zmc.scan_device(spec, d_axis, f, s, stream=stream,
                        events=(ev[i][0].cuda_event, ev[i][1].cuda_event))
        step_ev[i + 1].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    kernel_ms = np.array([a.elapsed_time(b) for a, b in ev])
    step_ms = np.array([step_ev[i].elapsed_time(step_ev[i + 1]) for i in range(steps)])
    ok = bool(torch.isfinite(f).all()) and bool(torch.isfinite(s).all())
    return dict(wall_s=wall, kernel_ms=kernel_ms, step_ms=step_ms, finite=ok,
                plan=zmc.plan(spec))


def batched_run(reps=1, count=512, seed=3):
    """The 512-scan batch in one captured graph vs the same scans launched
    back to back through the plain entry point (count, seed: another draw of
    the same shape distribution)."""
    import torch
    from paper_1910_01965_amd import workloads as wl
    from paper_1910_01965_amd import zmc
    specs = wl.batched_512(count=count, seed=seed)
    total = sum(sp.G * sp.samples for sp in specs)
    outs = [(torch.empty(sp.G, dtype=torch.float64, device="cuda"),
             torch.empty(sp.G, dtype=torch.float64, device="cuda")) for sp in specs]
    b = zmc.Batch(specs, outputs=outs)
    info = b.info()
    b.launch()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        b.launch()
    torch.cuda.synchronize()
    t_batch = (time.perf_counter() - t0) / reps
    b.close()
    axes = [zmc.axis_tensor(sp) for sp in specs]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for (f, s), sp, a in zip(outs, specs, axes):
        zmc.scan_device(sp, a, f, s)
    torch.cuda.synchronize()
    t_plain = time.perf_counter() - t0
    return {"value": total / t_batch, "unit": "samples/s", "seconds": t_batch,
            "plain_back_to_back": total / t_plain, "ratio_vs_plain": t_plain / t_batch,
            "scans": len(specs), "samples": total, "tiles": info["tiles"],
            "variants": info["variants"], "graph": bool(info["graph"]),
            "shape_seed": seed, "philox_seeds": f"0..{len(specs) - 1} (scan i has seed i)",
            "grid_pts_per_s": sum(sp.G for sp in specs) / t_batch,
            "roofline": mix_roofline(specs, t_batch)}


def serving_run(rate, duration, seed=7, budget=64 << 30, max_slots=0, compare_plain=False,
                admission="fifo", verify=0, slice_us=0):
    """Poisson arrivals of scans shaped like the 512-scan batch (family,
    N, grid size, samples drawn by default_rng(seed); request i has Philox
    seed i) into the continuous-batching server; latency = completion -
    submission.  Optionally the same request trace back to back through
    the plain entry point, and `verify` requests spread evenly over the
    trace re-run alone, one at a time, in a fresh server: a request's tiles
    depend only on the request, so each must equal its served result bit
    for bit.  Every other request is released once it has finished."""
    import torch
    from paper_1910_01965_amd import workloads as wl
    from paper_1910_01965_amd import zmc
    rng = np.random.default_rng(seed)
    t_arr = np.cumsum(rng.exponential(1.0 / rate, size=int(rate * duration * 3) + 16))
    t_arr = t_arr[t_arr < duration]
    n_req = len(t_arr)
    specs = [sp.with_(seed=i) for i, sp in enumerate(wl.batched_512(count=n_req, seed=seed))]
    total = sum(sp.G * sp.samples for sp in specs)
    srv = zmc.Server(hbm_budget_bytes=budget, max_slots=max_slots, admission=admission,
                     slice_us=slice_us)
    tickets = []
    t0 = time.perf_counter()
    for ta, sp in zip(t_arr, specs):
        now = time.perf_counter() - t0
        if ta > now:
            time.sleep(ta - now)
        tickets.append(srv.submit(sp))
    lat = []
    picked = set(np.linspace(0, n_req - 1, min(verify, n_req)).round().astype(int).tolist()) \
        if verify > 0 else set()
    served = {}
    t_say = time.perf_counter()
    for i, t in enumerate(tickets):
        lat.append(srv.wait(t)[1])
        if i in picked:
            served[i] = srv.outputs(t)
        else:
            srv.release(t)
        if time.perf_counter() - t_say > 15.0:  # progress of long runs
            log(f"  serving: {i + 1}/{n_req} requests done, {time.perf_counter() - t0:.0f} s")
            t_say = time.perf_counter()
    lat = np.array(lat)
    t_all = time.perf_counter() - t0
    stats = srv.stats()
    srv.close()
    out = {"rate_per_s": rate, "arrival_seconds": duration, "requests": n_req, "samples": total,
           "arrival_and_shape_seed": seed, "philox_seeds": "request i has seed i",
           "value": total / t_all, "unit": "samples/s", "wall_seconds": t_all,
           "latency_s": {"p50": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99)),
                         "mean": float(lat.mean()), "max": float(lat.max())},
           "slices": stats["slices"], "bytes_peak": stats["bytes_peak"],
           "budget_bytes": budget, "max_slots": max_slots if max_slots > 0 else 256,
           "admission": admission, "slice_us": slice_us, "roofline": mix_roofline(specs, t_all),
           "server_reported": {k: stats[k] for k in ("latency_p50_s", "latency_p99_s",
                                                     "latency_max_s", "samples_per_s")}}
    if served:
        alone = zmc.Server(hbm_budget_bytes=budget, max_slots=max_slots, admission=admission)
        equal = 0
        for i in sorted(served):
            t = alone.submit(specs[i])
            alone.wait(t)
            f, s = alone.outputs(t)
            torch.cuda.synchronize()
            equal += int(torch.equal(f, served[i][0]) and torch.equal(s, served[i][1]))
        alone.close()
        out["alone_rerun"] = {"requests": len(served), "bitwise_equal": equal,
                              "what": "requests spread evenly over the trace, re-run one at a time "
                                      "in a fresh server, vs their served f and sigma"}
        log(f"  re-run alone: {equal}/{len(served)} requests bitwise equal to their served results")
        del served
    if compare_plain:
        outs = [(torch.empty(sp.G, dtype=torch.float64, device="cuda"),
                 torch.empty(sp.G, dtype=torch.float64, device="cuda")) for sp in specs]
        axes = [zmc.axis_tensor(sp) for sp in specs]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for i, ((f, s), sp, a) in enumerate(zip(outs, specs, axes)):
            zmc.scan_device(sp, a, f, s)
            if (i + 1) % 1000 == 0:  # progress of long runs
                torch.cuda.synchronize()
                log(f"  plain launches: {i + 1}/{n_req}, {time.perf_counter() - t0:.0f} s")
        torch.cuda.synchronize()
        t_plain = time.perf_counter() - t0
        out["plain_back_to_back"] = total / t_plain
        # the server's device-busy throughput is bounded by arrivals only if it
        # ever idles; under overload it is total / (wall - first arrival gap)
        out["ratio_vs_plain"] = (total / t_all) / (total / t_plain)
    return out


def cpu_baseline(spec, points, seed=0):
    from oracle import oracle as zo
    idx = np.sort(np.random.default_rng(seed).choice(spec.G, points, replace=False)).astype(np.uint64)
    t0 = time.perf_counter()
    zo.scan(spec.with_(precision="fp64"), idx)
    dt = time.perf_counter() - t0
    model = ""
    try:
        with open("/proc/cpuinfo") as fh:
            model = next((l.split(":", 1)[1].strip() for l in fh if l.startswith("model name")), "")
    except OSError:
        pass
    full_s = spec.G * spec.samples / (points * spec.samples / dt)
    return {"value": points * spec.samples / dt, "unit": "samples/s", "cores": 1, "kind": "oracle",
            "sample": f"{points} seeded random grid points of {spec.name} (all {spec.samples} samples "
                      f"each, {points * spec.samples:.3g} samples), single-threaded FP64 oracle, "
                      f"{dt:.1f} s",
            "host": {"cpu": model, "logical_cpus": os.cpu_count()},
            "full_grid_one_core_s_extrapolated": full_s}


def cpu_baseline_threads(spec, points, seed=0):
    """The same oracle on the same seeded points, spread over the host's
    cores: one oracle call per slice of points from a pool of threads (the
    oracle's C entry point releases the interpreter lock and keeps no shared
    state; its arithmetic is unchanged)."""
    import concurrent.futures as cfut
    from oracle import oracle as zo
    idx = np.sort(np.random.default_rng(seed).choice(spec.G, points, replace=False)).astype(np.uint64)
    threads = max(1, min(16, os.cpu_count() or 1))
    parts = np.array_split(idx, 8 * threads)
    sp = spec.with_(precision="fp64")
    t0 = time.perf_counter()
    with cfut.ThreadPoolExecutor(threads) as ex:
        list(ex.map(lambda part: zo.scan(sp, part), parts))
    dt = time.perf_counter() - t0
    return {"value": points * spec.samples / dt, "unit": "samples/s", "cores": threads,
            "kind": "oracle", "seconds": dt,
            "sample": f"the same {points} points on {threads} threads"}


def cpu_full_grid_threads(spec):
    """The oracle over the whole grid on the host's cores (slices of points
    from a pool of threads, as cpu_baseline_threads): measured, not
    extrapolated."""
    import concurrent.futures as cfut
    from oracle import oracle as zo
    threads = max(1, min(16, os.cpu_count() or 1))
    parts = np.array_split(np.arange(spec.G, dtype=np.uint64), 64 * threads)
    sp = spec.with_(precision="fp64")
    t0 = time.perf_counter()
    with cfut.ThreadPoolExecutor(threads) as ex:
        list(ex.map(lambda part: zo.scan(sp, part), parts))
    dt = time.perf_counter() - t0
    return {"seconds": dt, "samples_per_s": spec.G * spec.samples / dt, "cores": threads,
            "kind": "oracle", "sample": f"all {spec.G} points of {spec.name} on {threads} threads"}


def cpu_baseline_others(seed=0):
    """The oracle on one host core for the other workloads: the whole
    1000-point plain FP64 scan, the 1e4-point subsample of the 1e8-point
    COSEXP grid and one seeded point of each of the 512 batch scans, each
    with its whole-workload single-core time extrapolated from the sample."""
    from oracle import oracle as zo
    from paper_1910_01965_amd import workloads as wl
    out = {}
    sp = wl.plain_fp64()
    t0 = time.perf_counter()
    zo.scan(sp)
    dt = time.perf_counter() - t0
    n = sp.G * sp.samples
    out[sp.name] = {"sample": "the whole scan", "samples": n, "seconds": dt, "samples_per_s": n / dt}
    sp = wl.cosexp_4p(precision="fp64")
    idx = wl.cosexp_subsample()
    t0 = time.perf_counter()
    zo.scan(sp, idx)
    dt = time.perf_counter() - t0
    n = len(idx) * sp.samples
    out["cosexp_4p_1e8pts_n4096"] = {
        "sample": f"the {len(idx)}-point subsample: np.random.default_rng(42).choice(10**8, "
                  f"10**4, replace=False), sorted", "samples": n, "seconds": dt,
        "samples_per_s": n / dt, "full_grid_one_core_s_extrapolated": sp.G * sp.samples / (n / dt)}
    rng = np.random.default_rng(seed)
    t_sum = t_full = 0.0
    n = 0
    for sp in wl.batched_512():
        g = np.array([rng.integers(0, sp.G)], dtype=np.uint64)
        t0 = time.perf_counter()
        zo.scan(sp.with_(precision="fp64"), g)
        dt = time.perf_counter() - t0
        t_sum += dt
        t_full += dt * sp.G
        n += sp.samples
    out["batched_512"] = {"sample": "one seeded point of each scan", "samples": n, "seconds": t_sum,
                          "samples_per_s": n / t_sum, "full_batch_one_core_s_extrapolated": t_full}
    return out


def paper_context():
    """The paper's own throughput on its own workloads and hardware, derived
    from the times it prints (Table 1, Table 2): context, not a target."""
    from paper_1910_01965_amd import replay
    t1 = {f"M4_N{N}": 1e8 * 1e4 / replay.PAPER_TABLE1[(4, N)][3] for N in (1, 2, 3, 4)}
    return {
        "note": "the paper's runs: other workloads and hardware; samples/s derived from its times",
        "table1": {"hardware": "1x NVIDIA Tesla V100 + Xeon Silver 4110",
                   "workload": "Eq. (2) on [0,10]^N, x_l in {0..99} (1e8 points at M=4), 1e4 samples",
                   "samples_per_s": t1},
        "table2": {"workload": "Eq. (4), N=6, 1e8 points x 1e5 samples in 100 batches of 1e6 points",
                   "v100_samples_per_s": 1e6 * 1e5 / replay.PAPER_TABLE2_V100_BATCH_S,
                   "cluster": "4x K40m + 2x K80 + 1x V100 over 3 nodes",
                   "cluster_samples_per_s": 1e8 * 1e5 / replay.PAPER_TABLE2_TOTAL_S}}


def copy_probe(nbytes=1 << 30, reps=3):
    """A plain device-to-device copy of known size: FETCH_SIZE / WRITE_SIZE
    of its dispatches calibrate the HBM counters against nbytes."""
    import torch
    src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(reps):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_probe_bytes": nbytes, "reps": reps}), flush=True)


def valu_probe(blocks=65536, iters=512, reps=3):
    """The VALU calibration load (eight independent FMA chains per lane):
    rocprofv3 VALU counters of its dispatches should read ~100 % issue-busy,
    which checks the busy fraction reported for the scan kernels."""
    import torch
    from paper_1910_01965_amd import zmc
    zmc.debug_valu_probe(blocks, iters)
    torch.cuda.synchronize()
    ms = []
    for _ in range(reps):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        zmc.debug_valu_probe(blocks, iters)
        b.record()
        torch.cuda.synchronize()
        ms.append(a.elapsed_time(b))
    fmas = 64.0 * iters * blocks * 256
    t = min(ms) / 1e3
    print(json.dumps({"valu_probe": {"blocks": blocks, "iters": iters, "fma_lanes": fmas,
                                     "ms": min(ms), "fma_lane_per_s": fmas / t,
                                     "vs_single_issue_peak": fmas / t / (VALU_PEAK / 2)}}), flush=True)


def dims_sweep(samples=1 << 12, steps=10, warmup=5):
    """Roofline fraction of the point-major kernels across the integration
    dimension, up to the descriptor's 16: GAUSS and SIN_SUM on a 1000 x 1000
    grid and COSEXP on 32^4 points, 4096 samples per point, both precisions;
    algorithmic operations per sample as in the main line, kernel time from
    HIP events after `warmup` scans (kernels of a few ms run slower until the
    device has been busy for a while).  One JSON line."""
    import torch
    from paper_1910_01965_amd import workloads as wl
    from paper_1910_01965_amd import zmc
    if not torch.cuda.is_available():
        raise SystemExit("no GPU visible")
    zmc.load()
    ax = np.linspace(0.1, 10.0, 1000)
    rows = []
    for fam, N in (("gauss", 3), ("gauss", 8), ("gauss", 12), ("gauss", 16), ("sin_sum", 8),
                   ("sin_sum", 16), ("cosexp", 16)):
        for prec in ("fp32", "fp64"):
            if fam == "gauss":
                sp = wl.ScanSpec("gauss", [ax, ax.copy()], np.zeros(N), np.ones(N), samples, 42, prec)
            elif fam == "sin_sum":
                sp = wl.ScanSpec("sin_sum", [np.linspace(0, 1, 1000)] * 2, np.zeros(N), np.ones(N),
                                 samples, 42, prec)
            else:
                hi = np.ones(N)
                hi[0] = 2.0
                sp = wl.ScanSpec("cosexp", [np.linspace(-1, 1, 32)] * 4, np.zeros(N), hi, samples, 42,
                                 prec)
            r = time_path(sp, steps, warmup)
            km = float(np.mean(r["kernel_ms"]))
            w = valu_ops_per_sample(fam, N)
            row = {"family": fam, "N": N, "precision": prec, "grid_points": sp.G, "samples": samples,
                   "kernel_ms": km, "samples_per_s": sp.G * samples / (km / 1e3),
                   "ops_per_sample": w, "frac": w * sp.G * samples / (km / 1e3) / VALU_PEAK,
                   "plan": r["plan"]}
            rows.append(row)
            log(f"{fam} N={N} {prec}: {km:.2f} ms, {row['samples_per_s']:.3g} samples/s, "
                f"frac {row['frac']:.3f}")
    print(json.dumps({"dims_sweep": rows, "peak": VALU_PEAK / 1e12, "unit": "T lane-op/s"}),
          flush=True)


def rate_probe(blocks=8192, iters=1024, reps=3):
    """Issue rate of each instruction form the scan kernels use
    (zmc_debug_rate_probe): lane-instructions per second, and that rate over
    one instruction per lane per clock on every CU (256 CUs x 64 lanes x
    2.4 GHz = 3.93e13/s)."""
    import torch
    from paper_1910_01965_amd import zmc
    unit = 256 * 64 * 2.4e9
    res = {}
    for op in zmc.RATE_OPS:
        zmc.debug_rate_probe(op, blocks, iters)
        torch.cuda.synchronize()
        ms = []
        for _ in range(reps):
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record()
            zmc.debug_rate_probe(op, blocks, iters)
            b.record()
            torch.cuda.synchronize()
            ms.append(a.elapsed_time(b))
        n = 64.0 * iters * blocks * 256
        rate = n / (min(ms) / 1e3)
        res[op] = {"ms": min(ms), "lane_insts_per_s": rate, "per_lane_per_clock_per_cu": rate / unit}
        log(f"rate probe {op}: {rate:.4g} lane-instructions/s = {rate / unit:.3f} x 64 lanes/clock/CU")
    print(json.dumps({"rate_probe": {"blocks": blocks, "threads": 256, "iters": iters,
                                     "insts_per_lane": 64 * iters, "ops": res}}), flush=True)


USER_GAUSS = ("template <typename T> __device__ T integrand(const T* y, const T* x, const T* p) {\n"
              "  return exp(-(x[0] * y[0] * y[0] + x[1] * y[1] * y[1] + y[2] * y[2]));\n}\n")


def user_run(spec, out):
    """The Gaussian bench workload as a run-time-compiled user integrand (the
    integrand written plainly, as a user would), FP32, FP64 and FP32 with
    approximate transcendentals, beside the compiled-in family; plus the
    one-time compile and load cost."""
    import torch
    from paper_1910_01965_amd import zmc
    res = {"source": USER_GAUSS}
    for key, prec, fast, steps, ref in (("fp32", "fp32", False, 5, out["value"]),
                                        ("fp64", "fp64", False, 2, out["fp64"]["value"]),
                                        ("fp32_fast_math", "fp32", True, 5, out["value"])):
        sp = spec.with_(family="user", source=USER_GAUSS, precision=prec, name=spec.name + "_user",
                        fast_math=fast)
        t0 = time.perf_counter()
        zmc.integrand(USER_GAUSS, fast)
        f, s = zmc.scan(sp.with_(axes=[a[:2] for a in sp.axes], samples=64))  # compiles (prec, N, M)
        torch.cuda.synchronize()
        first = time.perf_counter() - t0
        log(f"config user gauss {key}: first use (compile + load) {first:.2f} s, {steps} steps")
        r = time_path(sp, steps, 1)
        ms = r["wall_s"] * 1e3 / steps
        v = sp.G * sp.samples / (ms / 1e3)
        res[key] = {"samples_per_s": v, "ms_per_step": ms, "kernel_ms": float(np.mean(r["kernel_ms"])),
                    "vs_compiled_family": v / ref, "first_use_s": first}
        log(f"  {v:.4g} samples/s ({v / ref:.3f}x the compiled-in family)")
    return res


def end_to_end(spec, reps=3):
    """The same scan through the synchronous host-memory entry point (lists
    staged in, f and sigma copied back over PCIe into pageable arrays): the
    PCIe-inclusive rate, reported beside `value`, never as it."""
    from paper_1910_01965_amd import zmc
    zmc.scan_host(spec)
    best = float("inf")
    for _ in range(reps):
        t0 = time.perf_counter()
        zmc.scan_host(spec)
        best = min(best, time.perf_counter() - t0)
    log(f"end to end (host buffers): {best * 1e3:.2f} ms")
    return {"what": "zmc_scan with host buffers: staging, scan, f and sigma back (16 MB)",
            "ms": best * 1e3, "samples_per_s": spec.G * spec.samples / best}


def chunked_run(big=False):
    """Out-of-core scans into host memory.  The Boltzmann-shaped grid of the
    paper's Sec. 3.3 (momentum 30^3 x 10^3 values x 7 species = 1.89e8 points,
    a 5-dimensional integral; SIN_SUM over seven parameters stands in for the
    collision integrand, which the paper does not give), 1024 samples, FP32:
    device-only scan vs chunked into pageable and into pinned host arrays.
    `big`: a 2.1e9-point grid (34 GB of f and sigma) streamed in 2^24-point
    chunks."""
    import torch
    from paper_1910_01965_amd import workloads as wl
    from paper_1910_01965_amd import zmc
    spec = wl.boltzmann_shape()
    res = {"workload": spec.name, "grid_points": spec.G, "samples_per_point": spec.samples}
    r = time_path(spec, 2, 1)
    dev = r["wall_s"] / 2
    res["device_only_s"] = dev
    f = np.zeros(spec.G)
    s = np.zeros(spec.G)
    zmc.scan_chunked(spec, 0, f, s)
    t0 = time.perf_counter()
    zmc.scan_chunked(spec, 0, f, s)
    res["chunked_pageable_s"] = time.perf_counter() - t0
    del f, s
    fp = torch.empty(spec.G, dtype=torch.float64, pin_memory=True)
    sp = torch.empty(spec.G, dtype=torch.float64, pin_memory=True)
    t0 = time.perf_counter()
    zmc.scan_chunked(spec, 0, fp, sp)
    res["chunked_pinned_s"] = time.perf_counter() - t0
    del fp, sp
    for k in ("device_only_s", "chunked_pageable_s", "chunked_pinned_s"):
        res[k.replace("_s", "_pts_per_s")] = spec.G / res[k]
    log(f"chunked {spec.name}: device {dev:.3f} s, pageable {res['chunked_pageable_s']:.3f} s, "
        f"pinned {res['chunked_pinned_s']:.3f} s")
    if big:
        bspec = wl.ScanSpec("sin_sum", [np.linspace(0, 1, 2048), np.linspace(0, 1, 1024),
                                        np.linspace(0, 1, 1024)], np.zeros(2), np.ones(2), 16, 6, "fp32",
                            name="grid_2048x1024x1024_N2_n16")
        f = np.zeros(bspec.G)
        s = np.zeros(bspec.G)
        t0 = time.perf_counter()
        zmc.scan_chunked(bspec, 0, f, s)
        tb = time.perf_counter() - t0
        res["big"] = {"workload": bspec.name, "grid_points": bspec.G, "host_bytes": 16 * bspec.G,
                      "seconds": tb, "pts_per_s": bspec.G / tb, "finite": bool(np.isfinite(f).all())}
        log(f"chunked {bspec.name}: {tb:.2f} s for {bspec.G} points")
    return res


T_START = time.perf_counter()


def left(args):
    """Seconds left of the run's time budget."""
    return args.time_budget - (time.perf_counter() - T_START)


def fit_serving_window(asked, left_s, cap, plain, short_s, trace_samples, steady_s=8.0):
    """The arrival window to run: `asked` seconds, halved (down to 4 s) while
    the serving section would not fit in `left_s` seconds.  Its cost: serving
    the trace (never shorter than its arrivals) at `cap` samples/s, the same
    trace as plain launches at `plain` samples/s, the shortest-first run over
    `short_s` seconds of the same arrivals, the steady run and 30 s of
    margin."""
    short_cost = max(short_s, trace_samples(short_s) / cap)

    def cost(sec):
        tot = trace_samples(sec)
        return max(sec, tot / cap) + tot / plain + short_cost + 1.25 * steady_s + 30.0

    seconds = asked
    while seconds > 4.0 and cost(seconds) > left_s:
        seconds = max(4.0, seconds / 2)
    return seconds


def serving_section(args, out):
    """The serving workload as specified (Poisson arrivals at 200 req/s for
    --serve-seconds, seed 7, 64 GiB budget, arrival order) with the same
    trace back to back through the plain entry point; then shortest-first
    admission and a steady load at 0.7x capacity over short windows.  The
    arrival window shrinks, and says so, when the run's time budget would not
    hold it."""
    from paper_1910_01965_amd import workloads as wl
    cap = out["batched"]["value"] if "batched" in out else 6e11
    plain = out["batched"]["plain_back_to_back"] if "batched" in out else cap
    seconds = args.serve_seconds
    short_s = min(args.serve_short_seconds, seconds)

    def trace_samples(sec):
        rng = np.random.default_rng(7)
        t = np.cumsum(rng.exponential(1.0 / 200.0, size=int(200 * sec * 3) + 16))
        k = int(np.sum(t < sec))
        return sum(sp.G * sp.samples for sp in wl.batched_512(count=k, seed=7))

    asked = seconds
    seconds = fit_serving_window(asked, left(args), cap, plain, short_s, trace_samples,
                                 args.serve_steady_seconds)
    if seconds != asked:
        log(f"serving: {asked} s of arrivals would not fit the time budget; running {seconds} s")
    log(f"serving: 200 req/s for {seconds} s (arrival order), then the same trace as plain launches")
    over = serving_run(200.0, seconds, compare_plain=True, max_slots=args.serve_max_slots, verify=64)
    over["arrival_seconds_asked"] = asked
    log(f"serving overload: {over['value']:.4g} samples/s ({over['ratio_vs_plain']:.3f}x plain), "
        f"p50 {over['latency_s']['p50']:.3f} s, p99 {over['latency_s']['p99']:.3f} s")
    log(f"serving: 200 req/s for {short_s} s, shortest first")
    short = serving_run(200.0, short_s, admission="shortest", max_slots=args.serve_max_slots,
                        verify=16)
    short["ratio_vs_plain"] = short["value"] / over["plain_back_to_back"]
    log(f"serving overload, shortest first: {short['value']:.4g} samples/s, "
        f"p50 {short['latency_s']['p50']:.3f} s, p99 {short['latency_s']['p99']:.3f} s")
    mean_req = over["samples"] / max(1, over["requests"])
    steady_rate = 0.7 * cap / mean_req
    log(f"serving steady: {steady_rate:.1f} req/s for {args.serve_steady_seconds} s")
    steady = serving_run(steady_rate, args.serve_steady_seconds, seed=8,
                         max_slots=args.serve_max_slots)
    log(f"serving steady: p50 {steady['latency_s']['p50'] * 1e3:.1f} ms, "
        f"p99 {steady['latency_s']['p99'] * 1e3:.1f} ms")
    slots = args.serve_max_slots if args.serve_max_slots > 0 else 256
    out_s = {"overload_200_per_s": over, "overload_200_per_s_shortest_first": short,
             "steady_0p7_capacity": steady}
    if args.slice_sweep:
        # the same steady arrivals with slices sized for a target device time
        # (zmc_server_opts.slice_us; 0 = the default 4e9-sample slices)
        out_s["steady_slice_sweep"] = []
        for us in (int(x) for x in args.slice_sweep.split(",")):
            r = serving_run(steady_rate, args.serve_steady_seconds, seed=8,
                            max_slots=args.serve_max_slots, slice_us=us)
            log(f"serving steady, slice_us={us}: p50 {r['latency_s']['p50'] * 1e3:.1f} ms, "
                f"p99 {r['latency_s']['p99'] * 1e3:.1f} ms, {r['slices']} slices, "
                f"{r['value']:.4g} samples/s")
            out_s["steady_slice_sweep"].append(
                {"slice_us": us, "latency_s": r["latency_s"], "slices": r["slices"],
                 "value": r["value"], "requests": r["requests"], "rate_per_s": r["rate_per_s"]})
    out_s["what"] = (f"Poisson arrivals of 512-batch-shaped scans, 64 GiB budget, {slots} slots; "
                     "latency = completion - submission")
    return out_s


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--fp64-steps", type=int, default=5)
    ap.add_argument("--cpu-points", type=int, default=48000)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--no-configs", action="store_true")
    ap.add_argument("--no-serving", action="store_true")
    ap.add_argument("--no-chunked", action="store_true")
    ap.add_argument("--chunked-big", action="store_true",
                    help="also stream a 2.1e9-point grid (34 GB of host memory)")
    ap.add_argument("--grid-1e10", action="store_true",
                    help="also stream a 1e10-point grid (160 GB of results) in ranges")
    ap.add_argument("--serve-seconds", type=float, default=60.0,
                    help="arrival window of the specified serving run (arrival order)")
    ap.add_argument("--serve-short-seconds", type=float, default=4.0,
                    help="arrival window of the shortest-first run (at most --serve-seconds)")
    ap.add_argument("--serve-steady-seconds", type=float, default=8.0,
                    help="arrival window of the steady run at 0.7x capacity")
    ap.add_argument("--slice-sweep", default="",
                    help="comma-separated slice_us targets: the steady run again with each "
                         "(0 = the default slices); off by default")
    ap.add_argument("--serve-max-slots", type=int, default=0,
                    help="admitted requests at once (0 = the server's default, 256)")
    ap.add_argument("--time-budget", type=float, default=540.0,
                    help="seconds the whole run may take; the serving window shrinks and the "
                         "optional sections are skipped to stay within it")
    ap.add_argument("--copy-probe", action="store_true",
                    help="only run a plain 1 GiB device copy (HBM counter calibration)")
    ap.add_argument("--valu-probe", action="store_true",
                    help="only run the FMA-chain load (VALU counter calibration)")
    ap.add_argument("--dims-sweep", action="store_true",
                    help="only time the point-major kernels across N = 3..16 (roofline fractions)")
    ap.add_argument("--rate-probe", action="store_true",
                    help="only time the instruction-rate loads of the scan kernels' op mix")
    args = ap.parse_args()
    if args.copy_probe:
        copy_probe()
        return
    if args.valu_probe:
        valu_probe()
        return
    if args.rate_probe:
        rate_probe()
        return
    if args.dims_sweep:
        dims_sweep()
        return
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for --gpus {args.gpus}); the scan shards by "
              "grid-point ranges across GPUs with no exchange, which this library does not run.",
              file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1910_01965_amd import workloads as wl
    from paper_1910_01965_amd import zmc
    if not torch.cuda.is_available():
        raise SystemExit("no GPU visible")
    zmc.load()

    spec = wl.gauss_2p(precision="fp32")
    G, n = spec.G, spec.samples
    log(f"bench: {spec.name} fp32, warmup {args.warmup}, steps {args.steps}")
    r32 = time_path(spec, args.steps, args.warmup)
    ms_per_step = r32["wall_s"] * 1e3 / args.steps
    value = G * n / (ms_per_step / 1e3)
    kern_ms = float(np.mean(r32["kernel_ms"]))
    log(f"fp32: {ms_per_step:.3f} ms/step, kernel {kern_ms:.3f} ms, {value:.4g} samples/s")

    spec64 = spec.with_(precision="fp64")
    log(f"bench: {spec.name} fp64, steps {args.fp64_steps}")
    r64 = time_path(spec64, args.fp64_steps, 1)
    ms64 = r64["wall_s"] * 1e3 / args.fp64_steps
    kern64_ms = float(np.mean(r64["kernel_ms"]))
    log(f"fp64: {ms64:.3f} ms/step, kernel {kern64_ms:.3f} ms")

    from paper_1910_01965_amd import kernel_ids
    ids = kernel_ids.kernel_ids()
    roof = roofline(kernel_ids.GAUSS_F32_N3_POINT_MAJOR, spec.name, spec.family, spec.N, G * n, kern_ms,
                    ids, "k_point_major<Gauss<float,3>>")
    if roof["valu_counters"]:
        log(f"roofline: {roof['frac']:.3f} of the VALU peak by operation count, "
            f"{roof['valu_counters']['frac']:.3f} by executed VALU instructions")
    roof64 = roofline(kernel_ids.GAUSS_F64_N3_POINT_MAJOR, spec.name, spec.family, spec.N, G * n,
                      kern64_ms, ids, "k_point_major<Gauss<double,3>>")

    out = {
        "metric": METRIC, "value": value, "unit": "samples/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_per_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": spec.name, "grid_points": G, "samples_per_point": n, "N": spec.N,
                   "family": spec.family, "precision": "fp32 evaluation, fp64 merge", "seed": spec.seed,
                   "plan": r32["plan"]},
        "grid_pts_per_s": G / (ms_per_step / 1e3),
        "fp64": {"value": G * n / (ms64 / 1e3), "unit": "samples/s", "ms_per_step": ms64,
                 "grid_pts_per_s": G / (ms64 / 1e3), "steps": args.fp64_steps,
                 "kernel_ms": kern64_ms, "roofline": roof64},
        "latency_ms": {"p50": float(np.percentile(r32["step_ms"], 50)),
                       "p99": float(np.percentile(r32["step_ms"], 99)),
                       "what": "per-scan device time of back-to-back plain scans"},
        "roofline": roof,
        "finite": r32["finite"] and r64["finite"],
        "kernel_ms_median": float(np.median(r32["kernel_ms"])),
        "kernel_ms_min": float(np.min(r32["kernel_ms"])),
    }
    out["end_to_end"] = end_to_end(spec)
    if not args.no_configs:
        out["configs"] = {}
        # warm-up scans: a kernel of a few ms or less runs slower until the
        # device has been busy for a while
        for name, sp, steps, warm, kern, label in (
                ("plain_fp64_1000pts_n65536", wl.plain_fp64(), 20, 10, None, None),
                ("cosexp_4p_1e8pts_n4096_fp32", wl.cosexp_4p(precision="fp32"), 3, 1,
                 kernel_ids.COSEXP_F32_N2_POINT_MAJOR, "k_point_major<CosExp<float,2>>"),
                ("cosexp_4p_1e8pts_n4096_fp64", wl.cosexp_4p(precision="fp64"), 3, 1,
                 kernel_ids.COSEXP_F64_N2_POINT_MAJOR, "k_point_major<CosExp<double,2>>")):
            log(f"config {name}: {warm} warm-up, {steps} steps, then {steps} with timing events")
            w = time_path(sp, steps, warm, events=False)
            r = time_path(sp, steps, 0)
            ms = w["wall_s"] * 1e3 / steps
            km = float(np.mean(r["kernel_ms"]))
            c = out["configs"][name] = {
                "samples_per_s": sp.G * sp.samples / (ms / 1e3), "grid_pts_per_s": sp.G / (ms / 1e3),
                "ms_per_step": ms, "ms_per_step_with_events": r["wall_s"] * 1e3 / steps,
                "kernel_ms": km, "finite": w["finite"] and r["finite"], "seed": sp.seed,
                "plan": r["plan"],
                "kernel_ms_median": float(np.median(r["kernel_ms"])),
                "kernel_ms_min": float(np.min(r["kernel_ms"])), "steps": steps, "warmup": warm}
            if kern:
                c["roofline"] = roofline(kern, sp.name, sp.family, sp.N, sp.G * sp.samples, km, ids,
                                         label)
            log(f"  {c['samples_per_s']:.4g} samples/s, {ms:.3f} ms/step")
    if not args.no_batched:
        log("batched: 512 scans")
        out["batched"] = batched_run()
        log(f"batched: {out['batched']['value']:.4g} samples/s ({out['batched']['ratio_vs_plain']:.3f}x plain)")
        # the tile table was tuned on the 512-scan draw itself; a draw it has
        # not seen (128 scans, shape seed 5) checks that the gain carries over
        held = batched_run(count=128, seed=5)
        held["what"] = "128 scans of the same shape distribution, shape seed 5 (not tuned on)"
        out["batched"]["held_out_draw"] = held
        log(f"batched, held-out draw: {held['value']:.4g} samples/s ({held['ratio_vs_plain']:.3f}x plain)")
    if not args.no_cpu_baseline:
        log(f"cpu baseline: oracle on {args.cpu_points} points")
        out["cpu_baseline"] = cpu_baseline(spec, args.cpu_points)
        out["cpu_baseline"]["all_host_cores"] = cpu_baseline_threads(spec, args.cpu_points)
        log("cpu baseline: oracle on the other workloads")
        out["cpu_baseline"]["other_workloads"] = cpu_baseline_others()
    else:
        out["cpu_baseline"] = None
    if not args.no_serving:
        out["serving"] = serving_section(args, out)
        over = out["serving"]["overload_200_per_s"]
        out["latency_ms"]["serving_p50"] = over["latency_s"]["p50"] * 1e3
        out["latency_ms"]["serving_p99"] = over["latency_s"]["p99"] * 1e3
        out["latency_ms"]["serving_what"] = ("completion - submission of the served requests, "
                                             "200 req/s Poisson arrivals over the arrival window")
    skipped = []
    # after the serving section, so that its arrival window keeps the time budget
    if not args.no_cpu_baseline:
        if left(args) > 60:
            log("cpu baseline: oracle on the whole grid, all host cores")
            full = cpu_full_grid_threads(spec)
            full["vs_gpu_step"] = full["seconds"] / (ms_per_step / 1e3)
            out["cpu_baseline"]["full_grid_all_cores"] = full
            log(f"  {full['seconds']:.1f} s on {full['cores']} threads")
        else:
            skipped.append("cpu_baseline.full_grid_all_cores")
    if not args.no_configs:
        if left(args) > 30:
            out["configs"]["user_gauss_2p_1000x1000_n16384"] = user_run(spec, out)
        else:
            skipped.append("configs.user_gauss_2p_1000x1000_n16384")
    if not args.no_chunked:
        if left(args) > 30:
            out["chunked"] = chunked_run(args.chunked_big)
            if args.grid_1e10:
                out["chunked"]["grid_1e10"] = grid_1e10_run()
        else:
            skipped.append("chunked")
    if skipped:
        out["skipped_for_time"] = skipped
        log(f"skipped to stay within the time budget: {skipped}")
    out["paper_context"] = paper_context()
    out["bench_seconds"] = time.perf_counter() - T_START
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
