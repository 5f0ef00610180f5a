"""Batched scans (one captured hipGraph over many scans) vs the oracle, and
alone-vs-mix identity (needs an MI355X)."""
import sys

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


def _np(outs):
    return [(f.cpu().numpy(), s.cpu().numpy()) for f, s in outs]


def _mixed_specs():
    """Small scans of every family and precision, N = 1..8, ragged sample
    counts, grids on both sides of the point-major threshold."""
    rng = np.random.default_rng(11)
    out = []
    seed = 100
    for precision in ("fp32", "fp64"):
        for N in range(1, 9):
            for fam in ("sin_sum", "gauss", "cosexp", "linear", "const"):
                if fam == "cosexp" and N < 2:
                    continue
                L = int(rng.choice([3, 17, 40]))
                n = int(rng.choice([2, 3, 999, 1024, 4097]))
                if fam == "sin_sum":
                    axes, lo, hi = [np.linspace(0, 1, L)], np.zeros(N), np.linspace(1, 2, N)
                elif fam == "gauss":
                    M = min(2, N)
                    axes, lo, hi = [np.linspace(0.1, 10, L)] * M, np.zeros(N), np.ones(N)
                elif fam == "cosexp":
                    axes = [np.linspace(-1, 1, max(2, L // 8))] * 4
                    lo, hi = np.zeros(N), np.ones(N)
                    hi[0] = 2.0
                else:
                    axes, lo, hi = [np.arange(float(L))], -np.ones(N), np.ones(N)
                out.append(wl.ScanSpec(fam, axes, lo, hi, n, seed, precision))
                seed += 1
    return out


def _check_all(specs, outs, label):
    worst_f = worst_s = 0.0
    for sp, (f, s) in zip(specs, outs):
        G = sp.G
        idx = np.arange(G, dtype=np.uint64) if G <= 64 else np.sort(
            np.random.default_rng(sp.seed).choice(G, 64, replace=False)).astype(np.uint64)
        f_ref, s_ref = zo.scan(sp, idx)
        ii = idx.astype(np.int64)
        ef, es, _ = parity.check(f[ii], s[ii], f_ref, s_ref, sp.samples, sp.precision,
                                 f"{label} {sp.family} N={sp.N} G={G} n={sp.samples} {sp.precision}",
                                 small_n=sp.samples < 4096, volume=float(np.prod(sp.hi - sp.lo)))
        worst_f, worst_s = max(worst_f, ef.max()), max(worst_s, es.max())
    _say(f"{label}: {len(specs)} scans, worst err_f {worst_f:.3e}, worst err_sigma {worst_s:.3e}")


def test_mixed_batch_matches_oracle():
    specs = _mixed_specs()
    _say(f"batch of {len(specs)} mixed scans")
    outs = _np(_zmc().scan_batch(specs))
    _check_all(specs, outs, "mixed batch")


def test_small_tiles_and_sample_major_threshold():
    specs = _mixed_specs()[::3]
    for opts in (dict(pm_groups=5, sm_groups=64, pm_min_points=20), dict(pm_min_points=1 << 30)):
        _say(f"batch with {opts}")
        outs = _np(_zmc().scan_batch(specs, **opts))
        _check_all(specs, outs, f"batch {opts}")


def test_alone_equals_in_mix_bitwise():
    specs = _mixed_specs()
    mix = _np(_zmc().scan_batch(specs))
    for i in range(0, len(specs), 7):
        _say(f"alone scan {i}")
        alone = _np(_zmc().scan_batch([specs[i]]))[0]
        assert np.array_equal(alone[0], mix[i][0]) and np.array_equal(alone[1], mix[i][1]), i


def test_graph_replay_and_direct_launch_identical():
    import torch
    specs = _mixed_specs()[::2]
    zmc = _zmc()
    b = zmc.Batch(specs)
    info = b.info()
    assert info["graph"] == 1 and info["scans"] == len(specs)
    b.launch()
    torch.cuda.synchronize()
    first = _np(b.outputs)
    for rep in range(3):
        for f, s in b.outputs:
            f.fill_(np.nan)
            s.fill_(np.nan)
        torch.cuda.synchronize()
        b.launch()
        torch.cuda.synchronize()
        again = _np(b.outputs)
        for (fa, sa), (fb, sb) in zip(first, again):
            assert np.array_equal(fa, fb) and np.array_equal(sa, sb), rep
    b.close()
    for par in (False, True):
        direct = _np(zmc.scan_batch(specs, use_graph=False, parallel_variants=par))
        for (fa, sa), (fb, sb) in zip(first, direct):
            assert np.array_equal(fa, fb) and np.array_equal(sa, sb)


def test_batch_close_to_plain_scan():
    spec = wl.gauss_2p(points_per_axis=60, samples=1 << 13, precision="fp32")
    fb, sb = _np(_zmc().scan_batch([spec]))[0]
    f, s = _zmc().scan(spec)
    f, s = f.cpu().numpy(), s.cpu().numpy()
    assert np.allclose(fb, f, rtol=1e-6) and np.allclose(sb, s, rtol=1e-4)


def test_batched_512_shapes_sampled():
    """All 512 scans of the batch at full size (fp32) in one graph, 16 random
    points of every scan against the oracle."""
    specs = wl.batched_512()
    _say(f"batched_512: {len(specs)} scans")
    outs = _zmc().scan_batch(specs)
    worst = 0.0
    import torch
    for sp, (f, s) in zip(specs, outs):
        idx = np.sort(np.random.default_rng(sp.seed).choice(sp.G, 16, replace=False)).astype(np.uint64)
        ti = torch.from_numpy(idx.astype(np.int64)).cuda()
        fs, ss = f[ti].cpu().numpy(), s[ti].cpu().numpy()
        f_ref, s_ref = zo.scan(sp, idx)
        ef, _, _ = parity.check(fs, ss, f_ref, s_ref, sp.samples, "fp32", sp.name)
        worst = max(worst, ef.max())
    _say(f"batched_512 subset worst err_f {worst:.3e}")
