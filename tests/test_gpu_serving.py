"""The serving loop (continuous batching) on the GPU: every request's result
is bitwise the same alone and in the mix, matches the oracle, admission
respects the HBM budget, and requests that can never fit fail cleanly."""
import sys
import threading
import time

import numpy as np
import pytest

from oracle import oracle as zo
from paper_1910_01965_amd import workloads as wl

import parity

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1910_01965_amd import zmc
    zmc.load()
    return torch


def _zmc():
    from paper_1910_01965_amd import zmc
    return zmc


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _requests(count, seed=7, max_samples=1 << 14):
    """Request shapes of the 512-scan batch generator, sample counts capped so
    the test stays short; a few FP64 requests and a ragged one mixed in."""
    specs = wl.batched_512(count=count, seed=seed)
    out = []
    for i, sp in enumerate(specs):
        sp = sp.with_(samples=min(sp.samples, max_samples), seed=1000 + i)
        if i % 5 == 4:
            sp = sp.with_(precision="fp64")
        if i % 7 == 3:
            sp = sp.with_(samples=sp.samples + 3)
        out.append(sp)
    return out


def _alone(spec):
    f, s = _zmc().scan_batch([spec])[0]
    return f.cpu().numpy(), s.cpu().numpy()


def test_mix_equals_alone_and_oracle():
    """64 requests through the server, each re-run alone: bitwise equal; every
    fourth one against the oracle."""
    import torch
    zmc = _zmc()
    specs = _requests(64)
    srv = zmc.Server(max_slots=8, slice_tiles=512)
    tickets = []
    for i, sp in enumerate(specs):
        tickets.append(srv.submit(sp))
        if i % 6 == 5:
            time.sleep(0.01)  # arrivals while earlier requests are on the GPU
    lat = []
    for t in tickets:
        st, l = srv.wait(t)
        assert st == 0
        lat.append(l)
    stats = srv.stats()
    _say(f"serving: {stats}; latency p50 {np.median(lat) * 1e3:.1f} ms max {max(lat) * 1e3:.1f} ms")
    assert stats["completed"] == len(specs) and stats["failed"] == 0
    assert stats["slices"] > 1
    torch.cuda.synchronize()
    for i, (sp, t) in enumerate(zip(specs, tickets)):
        f, s = srv.outputs(t)
        f, s = f.cpu().numpy(), s.cpu().numpy()
        fa, sa = _alone(sp)
        assert np.array_equal(f, fa) and np.array_equal(s, sa), (i, sp.name)
        if i % 4 == 0:
            idx = np.sort(np.random.default_rng(i).choice(sp.G, min(sp.G, 6), replace=False))
            f_ref, s_ref = zo.scan(sp, idx.astype(np.uint64))
            parity.check(f[idx], s[idx], f_ref, s_ref, sp.samples, sp.precision, sp.name)
    srv.close()


@pytest.mark.parametrize("admission,max_wait_ms", [("fifo", 0), ("shortest", 0), ("shortest", 1)])
def test_budget_admission_and_oversized_request(admission, max_wait_ms):
    zmc = _zmc()
    specs = _requests(10, seed=8)
    plans = [zmc.batch_plan([sp]) for sp in specs]
    need = [p["workspace_bytes"] for p in plans]
    budget = int(max(need) * 1.5) + (1 << 20)
    _say(f"budget admission {admission} max_wait_ms={max_wait_ms}")
    srv = zmc.Server(hbm_budget_bytes=budget, max_slots=4, slice_tiles=256, admission=admission,
                     max_wait_ms=max_wait_ms)
    tickets = [srv.submit(sp) for sp in specs]
    for t in tickets:
        st, _ = srv.wait(t)
        assert st == 0
    stats = srv.stats()
    _say(f"budget {budget}: {stats}")
    assert stats["bytes_peak"] <= budget and stats["completed"] == len(specs)
    # a request whose own state exceeds the budget fails, the server carries on
    big = wl.gauss_2p(points_per_axis=1000, samples=1 << 16)
    t_big = srv.submit(big)
    t_ok = [srv.submit(sp) for sp in specs[:3]]
    st_big, _ = srv.wait(t_big)
    assert st_big == 2 and all(srv.wait(t)[0] == 0 for t in t_ok)
    f, s = srv.outputs(t_ok[1])
    fa, sa = _alone(specs[1])
    assert np.array_equal(f.cpu().numpy(), fa) and np.array_equal(s.cpu().numpy(), sa)
    srv.close()


def test_concurrent_submitters():
    zmc = _zmc()
    specs = _requests(16, seed=9, max_samples=1 << 12)
    srv = zmc.Server(max_slots=16)
    tickets = [None] * len(specs)

    def worker(k):
        for i in range(k, len(specs), 4):
            tickets[i] = srv.submit(specs[i])

    th = [threading.Thread(target=worker, args=(k,)) for k in range(4)]
    for t in th:
        t.start()
    for t in th:
        t.join()
    for t in tickets:
        assert srv.wait(t)[0] == 0
    for sp, t in zip(specs[::5], tickets[::5]):
        f, s = srv.outputs(t)
        fa, sa = _alone(sp)
        assert np.array_equal(f.cpu().numpy(), fa) and np.array_equal(s.cpu().numpy(), sa)
    srv.close()


def test_shutdown_drains_pending_requests():
    """Closing the server with requests still queued (2 slots, 16 requests)
    returns once all of them have run; their results equal their alone runs."""
    import torch
    zmc = _zmc()
    specs = _requests(16, seed=10, max_samples=1 << 13)
    srv = zmc.Server(max_slots=2)
    tickets = [srv.submit(sp) for sp in specs]
    srv.close()
    torch.cuda.synchronize()
    for sp, t in list(zip(specs, tickets))[::3]:
        f, s = srv.outputs(t)
        fa, sa = _alone(sp)
        assert np.array_equal(f.cpu().numpy(), fa) and np.array_equal(s.cpu().numpy(), sa)


def test_one_slot_serves_in_arrival_order():
    """With one slot the server admits requests in submission order: each
    completes after the one before it, poll agrees with wait, and the
    statistics count every request once (the pending and active gauges are
    refreshed by the scheduler loop after the wake-up, so they are not read
    here).  A request's completion time is its submission time plus its
    latency; the submission happens inside the submit call, whose start and
    end the host clock brackets (the library's clock is the same monotonic
    clock), so request i cannot have completed after request i + 1 if the
    earliest completion time of i is after the latest of i + 1."""
    zmc = _zmc()
    specs = _requests(8, seed=11, max_samples=1 << 14)
    srv = zmc.Server(max_slots=1)
    tickets, spans = [], []
    for sp in specs:
        t0 = time.monotonic()
        tickets.append(srv.submit(sp))
        spans.append((t0, time.monotonic()))
    lat = []
    for t in tickets:
        st, l = srv.wait(t)
        assert st == 0
        done, st2, l2 = srv.poll(t)
        assert done and st2 == 0 and l2 == l
        lat.append(l)
    earliest = [a + l for (a, _), l in zip(spans, lat)]
    latest = [b + l for (_, b), l in zip(spans, lat)]
    _say(f"one-slot latencies {['%.4f' % x for x in lat]}")
    assert all(earliest[i] <= latest[i + 1] for i in range(len(specs) - 1)), (earliest, latest)
    stats = srv.stats()
    assert stats["submitted"] == stats["admitted"] == stats["completed"] == len(specs)
    assert stats["failed"] == 0
    srv.close()


def _admission_order(admission, max_wait_ms):
    """One slot; a long request is admitted and holds it while eight more of
    distinct work are queued in an order that is not their size order.
    Returns (work, completion time) of the eight in submission order, the
    completion time being the host's submission time plus the latency the
    server reports.  Every result still equals its alone run bit for bit."""
    zmc = _zmc()
    srv = zmc.Server(max_slots=1, admission=admission, max_wait_ms=max_wait_ms)
    blocker = wl.gauss_2p(points_per_axis=1000, samples=1 << 16)
    sizes = [7, 2, 5, 1, 8, 3, 6, 4]
    specs = [wl.ScanSpec("gauss", [np.linspace(0.1, 10, 128 * k)] * 2, np.zeros(3), np.ones(3),
                         1 << 16, 500 + k, "fp32") for k in sizes]
    srv.submit(blocker)
    t_end = time.perf_counter() + 10.0
    while srv.stats()["admitted"] < 1 and time.perf_counter() < t_end:
        time.sleep(0.0005)
    assert srv.stats()["admitted"] == 1, "the long request was not admitted"
    tickets, t_sub = [], []
    for sp in specs:
        tickets.append(srv.submit(sp))
        t_sub.append(time.perf_counter())
    done = [ts + srv.wait(t)[1] for ts, t in zip(t_sub, tickets)]
    for sp, t in list(zip(specs, tickets))[::3]:
        f, s = srv.outputs(t)
        fa, sa = _alone(sp)
        assert np.array_equal(f.cpu().numpy(), fa) and np.array_equal(s.cpu().numpy(), sa)
    srv.close()
    return [(sp.G * sp.samples * sp.N, c) for sp, c in zip(specs, done)]


def test_shortest_first_admission():
    """Shortest first: once the long request frees the slot, the queued ones
    complete in ascending work.  With a 1 ms wait bound, below the long
    request's run time, every queued request is overdue when the slot frees,
    and the oldest-first rule restores arrival order."""
    pairs = _admission_order("shortest", 0)
    t0 = min(c for _, c in pairs)
    _say(f"shortest first: {[(w, round(c - t0, 4)) for w, c in pairs]}")
    by_work = [c for _, c in sorted(pairs)]
    assert all(b > a for a, b in zip(by_work, by_work[1:]))
    pairs = _admission_order("shortest", 1)
    t0 = min(c for _, c in pairs)
    _say(f"shortest first, 1 ms bound: {[round(c - t0, 4) for _, c in pairs]}")
    arrival = [c for _, c in pairs]
    assert all(b > a for a, b in zip(arrival, arrival[1:]))


def test_server_reports_latency_percentiles():
    """The server's own p50 / p99 / max latency equal those of the latencies
    it returned per request (same interpolation as numpy's default), and its
    throughput is the completed samples over the span from first submission
    to last completion."""
    zmc = _zmc()
    specs = _requests(24, seed=13, max_samples=1 << 12)
    srv = zmc.Server(max_slots=8)
    assert srv.stats()["latency_p50_s"] == 0.0 and srv.stats()["samples_per_s"] == 0.0
    tickets = [srv.submit(sp) for sp in specs]
    lat = np.array([srv.wait(t)[1] for t in tickets])
    st = srv.stats()
    srv.close()
    _say(f"server-reported p50 {st['latency_p50_s']:.6f} p99 {st['latency_p99_s']:.6f} "
         f"max {st['latency_max_s']:.6f} s, {st['samples_per_s']:.4g} samples/s")
    assert np.isclose(st["latency_p50_s"], np.percentile(lat, 50), rtol=1e-12, atol=0)
    assert np.isclose(st["latency_p99_s"], np.percentile(lat, 99), rtol=1e-12, atol=0)
    assert st["latency_max_s"] == lat.max()
    total = sum(sp.G * sp.samples for sp in specs)
    assert st["samples_completed"] == total
    assert 0.0 < st["samples_per_s"] <= total / lat.max()


def test_released_requests_hold_no_memory():
    """3000 small requests, each collected (outputs) or released once it has
    finished: the server tracks no ticket afterwards, the binding keeps no
    output, and device memory returns to where it started; a request still
    running cannot be released."""
    import torch
    zmc = _zmc()
    base = wl.ScanSpec("gauss", [np.linspace(0.5, 2.0, 16), np.linspace(0.5, 2.0, 16)],
                       np.zeros(3), np.ones(3), 64, 0, "fp32", name="gauss_16x16_n64")
    blocker = wl.gauss_2p(precision="fp32", samples=1 << 16)
    srv = zmc.Server(max_slots=1)
    t_block = srv.submit(blocker)
    t_next = srv.submit(base)
    with pytest.raises(zmc.ZmcError) as err:
        srv.release(t_next)  # waits behind the blocker for its only slot
    assert err.value.status == 5
    srv.wait(t_block)
    srv.wait(t_next)
    srv.release(t_block)
    srv.release(t_next)
    srv.close()
    torch.cuda.synchronize()
    mem0 = torch.cuda.memory_allocated()
    srv = zmc.Server(max_slots=64)
    live, peak = [], 0
    f_ref = s_ref = None
    for i in range(3000):
        live.append((i, srv.submit(base.with_(seed=i % 50))))
        if len(live) > 32:
            j, t = live.pop(0)
            assert srv.wait(t)[0] == 0
            if j % 50 == 7 and f_ref is None:
                f, s = srv.outputs(t)
                f_ref, s_ref = f.cpu().numpy(), s.cpu().numpy()
            elif j % 50 == 7:
                f, s = srv.outputs(t)
                assert np.array_equal(f.cpu().numpy(), f_ref) and np.array_equal(s.cpu().numpy(), s_ref)
            else:
                srv.release(t)
        peak = max(peak, torch.cuda.memory_allocated() - mem0)
    for _, t in live:
        assert srv.wait(t)[0] == 0
        srv.release(t)
    st = srv.stats()
    assert st["completed"] == 3000 and st["tickets"] == 0 and not srv._keep
    srv.close()
    torch.cuda.synchronize()
    _say(f"3000 released requests: peak {peak} B of outputs above the start, "
         f"{torch.cuda.memory_allocated() - mem0} B at the end")
    assert peak <= 34 * 2 * 16 * base.G * 2  # at most the live requests' f and sigma (+ cache rounding)
    assert torch.cuda.memory_allocated() - mem0 <= 2 * 16 * base.G * 4


def test_slice_duration_target():
    """slice_us sizes slices by device time (samples at the measured rate):
    the same requests run in many more, smaller slices at a 1 ms target than
    at a 16 ms one, with bitwise the same results."""
    import torch
    zmc = _zmc()
    specs = _requests(24, seed=9, max_samples=1 << 16)
    runs = {}
    for us in (1000, 16000):
        srv = zmc.Server(slice_us=us)
        tickets = [srv.submit(sp) for sp in specs]
        for t in tickets:
            assert srv.wait(t)[0] == 0
        stats = srv.stats()
        outs = [srv.outputs(t) for t in tickets]
        srv.close()
        torch.cuda.synchronize()
        runs[us] = (stats, [(f.cpu().numpy(), s.cpu().numpy()) for f, s in outs])
        _say(f"slice_us={us}: {stats['slices']} slices, next slice {stats['slice_samples_now']:.3g} "
             f"samples, {stats['samples_per_s']:.3g} samples/s")
    short, long_ = runs[1000][0], runs[16000][0]
    assert short["slices"] >= 2 * long_["slices"], (short["slices"], long_["slices"])
    assert long_["slice_samples_now"] >= 4 * short["slice_samples_now"]
    for (fa, sa), (fb, sb) in zip(runs[1000][1], runs[16000][1]):
        assert np.array_equal(fa, fb) and np.array_equal(sa, sb)
    for i in (0, 7):
        fa, sa = _alone(specs[i])
        assert np.array_equal(runs[1000][1][i][0], fa) and np.array_equal(runs[1000][1][i][1], sa)


def test_cancel_a_queued_request():
    """zmc_server_cancel: a request still queued finishes with ZMC_E_CANCELLED,
    its outputs untouched; an admitted or finished one cannot be cancelled;
    the other requests complete bitwise as alone."""
    import torch
    zmc = _zmc()
    big = wl.gauss_2p(points_per_axis=1000, samples=1 << 16, precision="fp32")
    small = _requests(5, seed=11, max_samples=1 << 12)
    _say("cancel: one slot, a large request ahead of five small ones")
    srv = zmc.Server(max_slots=1)
    t_big = srv.submit(big)
    deadline = time.time() + 30.0
    while srv.stats()["admitted"] < 1:               # the large request holds the slot
        assert time.time() < deadline
        time.sleep(0.001)
    assert srv.cancel(t_big) is False               # admitted: it runs to completion
    f3 = torch.full((small[3].G,), float("nan"), dtype=torch.float64, device="cuda")
    s3 = torch.full_like(f3, float("nan"))
    torch.cuda.synchronize()
    tickets = [srv.submit(sp) if i != 3 else srv.submit(sp, f=f3, sigma=s3)
               for i, sp in enumerate(small)]
    assert srv.cancel(tickets[3]) is True           # still queued behind the large one
    assert srv.wait(tickets[3])[0] == 6             # ZMC_E_CANCELLED
    with pytest.raises(zmc.ZmcError) as ei:
        srv.cancel(10 ** 9)
    assert ei.value.status == 1
    assert srv.wait(t_big)[0] == 0
    for i, t in enumerate(tickets):
        if i != 3:
            assert srv.wait(t)[0] == 0
    assert srv.cancel(tickets[0]) is False          # finished
    stats = srv.stats()
    assert stats["cancelled"] == 1 and stats["failed"] == 1 and stats["completed"] == 5
    outs = {i: srv.outputs(t) for i, t in enumerate(tickets) if i != 3}
    srv.close()
    torch.cuda.synchronize()
    assert torch.isnan(f3).all() and torch.isnan(s3).all()
    for i in (0, 4):
        fa, sa = _alone(small[i])
        assert np.array_equal(outs[i][0].cpu().numpy(), fa) and np.array_equal(outs[i][1].cpu().numpy(), sa)
