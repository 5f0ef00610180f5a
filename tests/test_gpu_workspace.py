"""Split-partial workspaces of zmc_scan_device are reused across calls without a
host wait (needs an MI355X): many scans with split partials, enqueued back to
back on one stream and interleaved on two streams with no synchronisation in
between, and with workspaces that grow past the number of buffers kept per
device, each equal bit for bit to the same scan run alone."""
import sys

import numpy as np
import pytest

from paper_1910_01965_amd import workloads as wl

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1910_01965_amd import zmc
    zmc.load()
    return torch


def _specs():
    # workspaces of 16 * splits * G bytes: 0.6 to 14 MB, growing call by call
    return [wl.gauss_2p(points_per_axis=100 + 90 * i, samples=8192 + 17 * i, precision="fp32")
            for i in range(6)]


KW = dict(mode="point_major", splits=4)


def _alone(spec):
    import torch
    from paper_1910_01965_amd import zmc
    d_axis = zmc.axis_tensor(spec)
    f = torch.empty(spec.G, dtype=torch.float64, device="cuda")
    s = torch.empty(spec.G, dtype=torch.float64, device="cuda")
    torch.cuda.synchronize()
    zmc.scan_device(spec, d_axis, f, s, stream=torch.cuda.current_stream(), **KW)
    torch.cuda.synchronize()
    return f.cpu().numpy().copy(), s.cpu().numpy().copy()


def _outputs(spec, copies):
    import torch
    from paper_1910_01965_amd import zmc
    d_axis = zmc.axis_tensor(spec)
    outs = [(torch.full((spec.G,), float("nan"), dtype=torch.float64, device="cuda"),
             torch.full((spec.G,), float("nan"), dtype=torch.float64, device="cuda"))
            for _ in range(copies)]
    return d_axis, outs


@pytest.mark.parametrize("streams", [1, 2])
def test_back_to_back_scans_reuse_workspaces(streams):
    import torch
    from paper_1910_01965_amd import zmc
    specs = _specs()
    print(f"workspace reuse, streams={streams}, {len(specs)} specs", flush=True)
    sys.stdout.flush()
    want = [_alone(sp) for sp in specs]
    rounds = 3
    bufs = [_outputs(sp, rounds) for sp in specs]
    ss = [torch.cuda.Stream() for _ in range(streams)]
    torch.cuda.synchronize()
    k = 0
    for r in range(rounds):                 # small to large, then again: buffers retire and return
        for i, sp in enumerate(specs):
            d_axis, outs = bufs[i]
            f, s = outs[r]
            zmc.scan_device(sp, d_axis, f, s, stream=ss[k % streams], **KW)
            k += 1
    torch.cuda.synchronize()
    for i in range(len(specs)):
        for r in range(rounds):
            f, s = bufs[i][1][r]
            assert np.array_equal(f.cpu().numpy(), want[i][0]), (i, r)
            assert np.array_equal(s.cpu().numpy(), want[i][1]), (i, r)


@pytest.mark.parametrize("splits", [1, 4])
def test_lists_staged_by_the_call(splits):
    """zmc_scan_device with d_axis_vals = NULL stages desc->axis_vals itself:
    back-to-back calls give the results of the call with device lists, bit
    for bit."""
    import torch
    from paper_1910_01965_amd import zmc
    spec = wl.gauss_2p(points_per_axis=150, samples=4099, precision="fp32")
    print(f"lists staged by the call, splits={splits}", flush=True)
    kw = dict(mode="point_major", splits=splits)
    d_axis = zmc.axis_tensor(spec)
    f0 = torch.empty(spec.G, dtype=torch.float64, device="cuda")
    s0 = torch.empty_like(f0)
    torch.cuda.synchronize()
    zmc.scan_device(spec, d_axis, f0, s0, stream=torch.cuda.current_stream(), **kw)
    outs = [(torch.full_like(f0, float("nan")), torch.full_like(s0, float("nan"))) for _ in range(3)]
    for f, s in outs:
        zmc.scan_device(spec, None, f, s, stream=torch.cuda.current_stream(), **kw)
    torch.cuda.synchronize()
    for f, s in outs:
        assert torch.equal(f, f0) and torch.equal(s, s0)


def test_workspace_allocations_are_logged():
    """ZMC_LOG=2 reports each workspace buffer the cache allocates (a child
    process, since the library reads the level once)."""
    import os
    import subprocess
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    code = ("import torch\n"
            "from paper_1910_01965_amd import zmc, workloads as wl\n"
            "spec = wl.gauss_2p(points_per_axis=100, samples=4099)\n"
            "for _ in range(3):\n"
            "    zmc.scan(spec, mode='point_major', splits=4)\n"
            "torch.cuda.synchronize()\n")
    print("workspace logging in a child process", flush=True)
    r = subprocess.run([sys.executable, "-c", code], cwd=root, env=dict(os.environ, ZMC_LOG="2"),
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stderr[-2000:]
    lines = [ln for ln in r.stderr.splitlines() if ln.startswith("[zmc] workspace: new")]
    assert len(lines) == 1, r.stderr[-2000:]        # the three scans share one buffer


def test_mixed_sizes_settle_on_few_buffers():
    """Back-to-back scans whose workspaces range over 0.16..16 MB in shuffled
    order: buffers come in power-of-two sizes, so a larger one serves later
    smaller calls and the cache allocates at most one buffer per size class
    (1, 2, 4, 8, 16 MiB) instead of one per call."""
    import os
    import subprocess
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    code = ("import numpy as np, torch\n"
            "from paper_1910_01965_amd import zmc, workloads as wl\n"
            "rng = np.random.default_rng(5)\n"
            "for p in rng.integers(50, 500, size=40):\n"
            "    zmc.scan(wl.gauss_2p(points_per_axis=int(p), samples=1029), mode='point_major',"
            " splits=4)\n"
            "torch.cuda.synchronize()\n")
    print("workspace sizes of a shuffled mix in a child process", flush=True)
    r = subprocess.run([sys.executable, "-c", code], cwd=root, env=dict(os.environ, ZMC_LOG="2"),
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stderr[-2000:]
    new = [ln for ln in r.stderr.splitlines() if ln.startswith("[zmc] workspace: new")]
    assert 1 <= len(new) <= 5, "\n".join(new)
