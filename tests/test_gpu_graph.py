"""A caller's HIP graph may hold zmc_scan_device (needs an MI355X): the scan,
with and without split partials (stream-ordered workspace), is captured into
a torch CUDA graph; every replay, with eager work and synchronisations in
between, equals the eager scan bit for bit."""
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


@pytest.mark.parametrize("splits", [1, 4])
def test_scan_captured_in_a_graph(splits):
    import torch
    from paper_1910_01965_amd import zmc
    spec = wl.gauss_2p(points_per_axis=200, samples=4099, precision="fp32")
    print(f"graph capture, splits={splits}", flush=True)
    sys.stdout.flush()
    d_axis = zmc.axis_tensor(spec)
    f = torch.empty(spec.G, dtype=torch.float64, device="cuda")
    s = torch.empty(spec.G, dtype=torch.float64, device="cuda")
    kw = dict(mode="point_major", splits=splits)
    side = torch.cuda.Stream()
    with torch.cuda.stream(side):
        zmc.scan_device(spec, d_axis, f, s, stream=side, **kw)   # warm-up outside the capture
    torch.cuda.synchronize()
    f_eager, s_eager = f.cpu().numpy().copy(), s.cpu().numpy().copy()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        zmc.scan_device(spec, d_axis, f, s, stream=torch.cuda.current_stream(), **kw)
    for rep in range(4):
        f.fill_(float("nan"))
        s.fill_(float("nan"))
        junk = torch.ones(1 << 20, device="cuda") * rep   # eager work between replays
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert np.array_equal(f.cpu().numpy(), f_eager), rep
        assert np.array_equal(s.cpu().numpy(), s_eager), rep
        del junk
    g.reset()


def test_capture_refuses_lists_left_in_host_memory():
    """Under capture the parameter lists must already be on the device: a call
    that would stage them from host memory is refused before it records
    anything, and the capture goes on."""
    import torch
    from paper_1910_01965_amd import zmc
    spec = wl.gauss_2p(points_per_axis=100, samples=1029, precision="fp32")
    print("capture with host lists", flush=True)
    sys.stdout.flush()
    d_axis = zmc.axis_tensor(spec)
    f = torch.empty(spec.G, dtype=torch.float64, device="cuda")
    s = torch.empty(spec.G, dtype=torch.float64, device="cuda")
    side = torch.cuda.Stream()
    with torch.cuda.stream(side):
        zmc.scan_device(spec, d_axis, f, s, stream=side)   # warm-up outside the capture
    torch.cuda.synchronize()
    f_eager = f.cpu().numpy().copy()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        with pytest.raises(zmc.ZmcError) as ei:
            zmc.scan_device(spec, None, f, s, stream=torch.cuda.current_stream())
        zmc.scan_device(spec, d_axis, f, s, stream=torch.cuda.current_stream())
    assert ei.value.status == 1 and "capture" in str(ei.value)
    f.fill_(float("nan"))
    torch.cuda.synchronize()
    g.replay()
    torch.cuda.synchronize()
    assert np.array_equal(f.cpu().numpy(), f_eager)
    g.reset()
