"""Host builds of pieces of the HIP path (no GPU): both Philox paths of the
kernels give the same blocks, and the generic path matches the oracle."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(ROOT, "paper_1910_01965_amd", "csrc")


@pytest.fixture(scope="module")
def hipcc():
    path = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(path):
        pytest.skip("hipcc not available")
    return path


def test_point_major_philox_equals_generic(hipcc, tmp_path):
    exe = str(tmp_path / "philox_paths")
    subprocess.run([hipcc, "-x", "hip", "--offload-arch=gfx950", "-O2", "-I", CSRC,
                    "-I", os.path.join(ROOT, "include"),
                    os.path.join(HERE, "cpu_checks", "philox_paths.cpp"), "-o", exe], check=True)
    out = subprocess.run([exe], capture_output=True, text=True)
    bad, total = (int(t) for t in out.stdout.split())
    assert total == 200000 and bad == 0 and out.returncode == 0


def test_fp64_exp2_sine_cosine_against_long_double(hipcc, tmp_path):
    """The FP64 2^t of the COSEXP kernels and the FP64 sine and cosine of the
    SIN_SUM and COSEXP kernels, built for the host: within a few units in the
    last place of long-double libm over dense grids, and exact at the edges."""
    exe = str(tmp_path / "fp64_math")
    subprocess.run([hipcc, "-x", "hip", "--offload-arch=gfx950", "-O2", "-I", CSRC,
                    "-I", os.path.join(ROOT, "include"),
                    os.path.join(HERE, "cpu_checks", "fp64_math.cpp"), "-o", exe], check=True)
    out = subprocess.run([exe], capture_output=True, text=True)
    assert out.returncode == 0, out.stderr
    err_exp2, err_sin, err_cos, bad = out.stdout.split()
    assert float(err_exp2) < 4e-16 and float(err_sin) < 4e-16 and float(err_cos) < 4e-16, out.stdout
    assert int(bad) == 0, out.stdout
