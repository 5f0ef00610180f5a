"""The C ABI from plain C on the GPU (needs an MI355X): tests/c/zmc_abi_check
runs host-memory scans in both precisions, a range scan, a run-time user
integrand, and (with hipMalloc'd buffers) a device scan, a three-scan batch
and the server, checked against the oracle linked into it and against each
other bit for bit."""
import os
import subprocess

import pytest

pytestmark = pytest.mark.gpu

EXE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "c", "zmc_abi_check")


def test_c_program_on_the_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    if not os.path.exists(EXE):
        pytest.fail("tests/c/zmc_abi_check is not built (run __graft_entry__.build())")
    print("running tests/c/zmc_abi_check --gpu", flush=True)
    r = subprocess.run([EXE, "--gpu"], capture_output=True, text=True, timeout=100)
    print(r.stdout, flush=True)
    assert r.returncode == 0, r.stdout + r.stderr
    assert r.stdout.strip().endswith("passed")
