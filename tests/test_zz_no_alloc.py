"""The allocation-free scan (zmc_scan_device_noalloc) against the allocating
zmc_scan_device and the oracle, through the C ABI (needs an MI355X).

Both entry points plan the same way and run the same kernels, so their f and
sigma must agree bit for bit; the oracle checks sampled points to the usual
bars (FP64 1e-12; FP32 2e-5 on f, 1e-3 on sigma).  Two calls run in a row on
one stream, the second on a smaller scan, so the second reuses the scratch
that the first left behind.
"""
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
    zmc.load()  # raises when the HIP library is missing: no fallback
    return torch


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _outputs(G):
    import torch
    return (torch.full((G,), float("nan"), dtype=torch.float64, device="cuda"),
            torch.full((G,), float("nan"), dtype=torch.float64, device="cuda"))


def test_noalloc_equals_scan_device_on_two_calls():
    import torch
    from paper_1910_01965_amd import zmc
    # first: point-major FP32 with split partials (a ragged last group);
    # second, smaller: sample-major FP64 with split partials
    big = wl.gauss_2p(points_per_axis=320, samples=4099, precision="fp32")
    small = wl.plain_fp64().with_(axes=[np.linspace(0, 1, 100)], name="plain_fp64_100pts")
    specs = (big, small)
    for sp in specs:
        pl = zmc.plan(sp)
        _say(f"noalloc: {sp.name} {sp.precision} plan {pl}")
        assert pl["splits"] > 1 and 0 < pl["workspace_bytes"] <= zmc.NOALLOC_SCRATCH_BYTES
    stream = torch.cuda.current_stream()
    axes = [zmc.axis_tensor(sp) for sp in specs]
    free = [_outputs(sp.G) for sp in specs]
    for sp, a, (f, s) in zip(specs, axes, free):  # back to back, larger first
        zmc.scan_device_noalloc(sp, a, f, s, stream=stream)
    alloc = [_outputs(sp.G) for sp in specs]
    for sp, a, (f, s) in zip(specs, axes, alloc):
        zmc.scan_device(sp, a, f, s, stream=stream)
    torch.cuda.synchronize()
    for sp, (f1, s1), (f0, s0) in zip(specs, free, alloc):
        f1, s1, f0, s0 = (t.cpu().numpy() for t in (f1, s1, f0, s0))
        _say(f"noalloc: {sp.name}: compare {sp.G} points with zmc_scan_device")
        assert np.all(np.isfinite(f1)) and np.all(np.isfinite(s1))
        assert np.array_equal(f1, f0) and np.array_equal(s1, s0), sp.name
        idx = np.sort(np.random.default_rng(5).choice(sp.G, min(sp.G, 100), replace=False))
        f_ref, s_ref = zo.scan(sp.with_(precision="fp64"), idx.astype(np.uint64))
        _, _, msg = parity.check(f1[idx], s1[idx], f_ref, s_ref, sp.samples, sp.precision,
                                 label=f"noalloc {sp.name}", small_n=False, volume=1.0)
        _say(msg)


def test_noalloc_refuses_partials_beyond_its_scratch():
    import torch
    from paper_1910_01965_amd import zmc
    sp = wl.gauss_2p(precision="fp32")  # 1e6 points x 9 pieces: 144 MB of partials
    pl = zmc.plan(sp)
    _say(f"noalloc refusal: {sp.name} plan {pl}")
    assert pl["workspace_bytes"] > zmc.NOALLOC_SCRATCH_BYTES
    a = zmc.axis_tensor(sp)
    f, s = _outputs(sp.G)
    torch.cuda.synchronize()
    with pytest.raises(zmc.ZmcError) as ei:
        zmc.scan_device_noalloc(sp, a, f, s)
    assert ei.value.status == 2 and "scratch" in str(ei.value)
    torch.cuda.synchronize()
    assert bool(torch.isnan(f).all()) and bool(torch.isnan(s).all())  # nothing was launched
