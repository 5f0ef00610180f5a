"""The oracle's command-line front end (no GPU): it parses a plain-text scan
description and prints the same f and sigma as the library binding."""
import os
import subprocess

import numpy as np
import pytest

from oracle import build as ob
from oracle import oracle as zo
from paper_1910_01965_amd.workloads import ScanSpec


@pytest.fixture(scope="module")
def cli():
    if not os.path.exists(ob.CLI):
        ob.build_cli()
    return ob.CLI


def _write(path, spec):
    with open(path, "w") as fh:
        fh.write(f"# {spec.family} scan\nfamily {spec.family}\nsamples {spec.samples}\nseed {spec.seed}\n")
        for lo, hi in zip(spec.lo, spec.hi):
            fh.write(f"box {float(lo)!r} {float(hi)!r}\n")
        for a in spec.axes:
            fh.write("axis " + " ".join(repr(float(v)) for v in a) + "\n")


def _run(cli, path, *idx):
    out = subprocess.run([cli, path, *[str(i) for i in idx]], capture_output=True, text=True, check=True)
    rows = np.array([[float(x) for x in l.split()] for l in out.stdout.splitlines()])
    return rows[:, 0].astype(np.int64), rows[:, 1], rows[:, 2]


@pytest.mark.parametrize("spec", [
    ScanSpec("gauss", [np.linspace(0.1, 10, 4), np.linspace(0.3, 2, 3)], np.zeros(3), np.ones(3), 999, 7),
    ScanSpec("sin_sum", [np.arange(5.0)], np.zeros(2), np.full(2, 10.0), 1001, 18446744073709551557),
    ScanSpec("cosexp", [np.linspace(-1, 1, 3)] * 4, np.zeros(2), np.array([2.0, 1.0]), 64, 3),
], ids=["gauss", "sin_sum", "cosexp"])
def test_cli_matches_binding(cli, tmp_path, spec):
    path = str(tmp_path / "scan.txt")
    _write(path, spec)
    g, f, s = _run(cli, path)
    fr, sr = zo.scan(spec)
    assert np.array_equal(g, np.arange(spec.G)) and np.array_equal(f, fr) and np.array_equal(s, sr)
    g, f, s = _run(cli, path, spec.G - 1, 0)
    assert list(g) == [spec.G - 1, 0] and f[0] == fr[-1] and s[1] == sr[0]


def test_cli_rejects_bad_input(cli, tmp_path):
    path = str(tmp_path / "bad.txt")
    with open(path, "w") as fh:
        fh.write("family nope\nsamples 10\nbox 0 1\n")
    assert subprocess.run([cli, path], capture_output=True).returncode == 1
    with open(path, "w") as fh:
        fh.write("family gauss\nsamples 1\nbox 0 1\n")
    assert subprocess.run([cli, path], capture_output=True).returncode == 2
