"""The oracle under AddressSanitizer and UndefinedBehaviorSanitizer (host
code only, gcc): its command-line front end runs scans of every family,
edge shapes and subsets without a sanitizer report and prints exactly what
the regular build prints."""
import os
import shutil
import subprocess

import numpy as np
import pytest

from oracle import build as ob
from paper_1910_01965_amd.workloads import ScanSpec

SPECS = [
    ScanSpec("gauss", [np.linspace(0.1, 10, 5), np.linspace(0.3, 2, 4)], np.zeros(3), np.ones(3), 1001, 7),
    ScanSpec("sin_sum", [], np.zeros(4), np.ones(4), 4099, 1),                       # M = 0
    ScanSpec("cosexp", [np.linspace(-1, 1, 2)] * 4, np.zeros(5), np.array([2.0, 1, 1, 1, 1]), 3, 2),
    ScanSpec("linear", [np.arange(1.0)], -np.ones(8), np.ones(8), 2, 18446744073709551615),
    ScanSpec("const", [np.arange(2.0)] * 16, np.zeros(1), np.ones(1), 5, 3),         # 16 axes
]


def _write(path, spec):
    with open(path, "w") as fh:
        fh.write(f"family {spec.family}\nsamples {spec.samples}\nseed {spec.seed}\n")
        for lo, hi in zip(spec.lo, spec.hi):
            fh.write(f"box {float(lo)!r} {float(hi)!r}\n")
        for a in spec.axes:
            fh.write("axis " + " ".join(repr(float(v)) for v in a) + "\n")


@pytest.fixture(scope="module")
def binaries(tmp_path_factory):
    if shutil.which("gcc") is None:
        pytest.skip("gcc not available")
    d = tmp_path_factory.mktemp("san")
    san = str(d / "cli_san")
    subprocess.run(["gcc", "-std=c99", "-O1", "-g", "-fno-omit-frame-pointer",
                    "-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-I", ob.HERE,
                    ob.CLI_SRC, ob.SRC, "-o", san, "-lm"], check=True)
    plain = ob.build_cli(out=str(d / "cli"))
    return san, plain


@pytest.mark.parametrize("spec", SPECS, ids=lambda s: f"{s.family}-M{s.M}-N{s.N}")
def test_oracle_clean_under_sanitizers(binaries, tmp_path, spec):
    san, plain = binaries
    path = str(tmp_path / "scan.txt")
    _write(path, spec)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1")
    for extra in ([], [str(spec.G - 1), "0"]):
        a = subprocess.run([san, path, *extra], capture_output=True, text=True, env=env)
        b = subprocess.run([plain, path, *extra], capture_output=True, text=True)
        assert a.returncode == 0, a.stderr[-2000:]
        assert "runtime error" not in a.stderr and "Sanitizer" not in a.stderr, a.stderr[-2000:]
        assert a.stdout == b.stdout and a.stdout
