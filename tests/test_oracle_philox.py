"""Pins of the oracle's random words (CPU only).

The paper names no generator; the scan uses Philox4x32-10 (Salmon et al.,
SC'11) keyed by the seed with counter (word block, grid index).  The oracle's
Philox is pinned to (i) the published Random123 known-answer vectors and
(ii) two independent open-source implementations compiled here from their
headers, whose (seed, subsequence, offset) stream convention is the one the
scan uses: word w of grid point g is the w-th word of subsequence g.
"""
import os
import shutil
import subprocess

import numpy as np
import pytest

from oracle import oracle as zo
from paper_1910_01965_amd.workloads import ScanSpec

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")

# (seed, grid index g, first word w0, count): small and large g (above 2^32),
# word blocks above 2^32, a 64-bit seed.
CASES = [
    (42, 0, 0, 64),
    (42, 999, 0, 64),
    (7, 123456789, 5, 40),
    (0xDEADBEEFCAFEF00D, (1 << 33) + 17, 12, 24),
    (1, 3, (1 << 34) + 8, 16),
    (0xFFFFFFFFFFFFFFFF, (1 << 64) - 1, 4 * ((1 << 32) - 1), 16),
]


def _kat_rows():
    rows = []
    with open(os.path.join(GOLDEN, "philox4x32_10_kat.txt")) as fh:
        for line in fh:
            if line.startswith("#") or not line.strip():
                continue
            v = [int(t, 16) for t in line.split()]
            rows.append((v[0:4], v[4:6], v[6:10]))
    return rows


def test_published_known_answers():
    rows = _kat_rows()
    assert len(rows) == 3
    for ctr, key, out in rows:
        assert zo.philox(ctr, key) == out


def test_word_is_lane_of_block():
    # word w of point g is lane w mod 4 of the block with counter (b, g)
    for seed, g, w0, count in CASES[:4]:
        for w in range(w0, w0 + count):
            b = w // 4
            blk = zo.philox([b & 0xFFFFFFFF, b >> 32, g & 0xFFFFFFFF, g >> 32],
                            [seed & 0xFFFFFFFF, seed >> 32])
            assert zo.word(seed, g, w) == blk[w % 4]


def _run_generator(exe, lines):
    inp = "".join(f"{a} {b} {c} {d}\n" for a, b, c, d in lines)
    out = subprocess.run([exe], input=inp, capture_output=True, text=True, check=True).stdout
    return [int(t, 16) for t in out.split()]


@pytest.fixture(scope="module")
def aten_exe(tmp_path_factory):
    import torch
    inc = os.path.join(os.path.dirname(torch.__file__), "include")
    cxx = shutil.which("g++")
    if cxx is None or not os.path.isdir(inc):
        pytest.skip("g++ or the ATen headers are not available")
    exe = str(tmp_path_factory.mktemp("aten") / "philox_aten")
    subprocess.run([cxx, "-std=c++17", "-O1", "-I", inc,
                    os.path.join(GOLDEN, "philox_stream_aten.cpp"), "-o", exe], check=True)
    return exe


def build_rocrand_exe(outdir):
    """Compile the rocRAND cross-check generator into outdir; None if no toolchain."""
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc) or not os.path.exists(
            "/opt/rocm/include/rocrand/rocrand_philox4x32_10.h"):
        return None
    exe = os.path.join(str(outdir), "philox_rocrand")
    subprocess.run([hipcc, "-x", "hip", "--offload-arch=gfx950", "-O1", "-I", "/opt/rocm/include",
                    os.path.join(GOLDEN, "philox_stream_rocrand.cpp"), "-o", exe], check=True)
    return exe


@pytest.fixture(scope="module")
def rocrand_exe(tmp_path_factory):
    exe = build_rocrand_exe(tmp_path_factory.mktemp("rocrand"))
    if exe is None:
        pytest.skip("hipcc or the rocRAND headers are not available")
    return exe


def test_stream_matches_aten(aten_exe):
    # ATen's offset counts 128-bit blocks: start at block w0 / 4 (w0 % 4 == 0)
    lines = [(s, g, w0 // 4, c) for s, g, w0, c in CASES if w0 % 4 == 0]
    words = _run_generator(aten_exe, lines)
    i = 0
    for s, g, off, c in lines:
        ref = words[i:i + c]
        i += c
        got = [zo.word(s, g, 4 * off + j) for j in range(c)]
        assert got == ref, (s, g, off)


def test_stream_matches_rocrand(rocrand_exe):
    # rocRAND's offset counts words
    words = _run_generator(rocrand_exe, CASES)
    i = 0
    for s, g, w0, c in CASES:
        ref = words[i:i + c]
        i += c
        got = [zo.word(s, g, w0 + j) for j in range(c)]
        assert got == ref, (s, g, w0)


def test_sample_coordinates_follow_word_order(rocrand_exe):
    # LINEAR on [0,1]^2: v_s = u_{2s} + u_{2s+1} with u = (r + 1/2) 2^-32; the
    # sum of two such values is exact in FP64, so 2^32 v_s - 1 is exactly the
    # sum of words 2s and 2s+1 of the rocRAND stream of subsequence g.
    g, seed, n = 5, 42, 32
    spec = ScanSpec("linear", [np.arange(10.0)], np.zeros(2), np.ones(2), n, seed)
    v = zo.values(spec, g)
    words = _run_generator(rocrand_exe, [(seed, g, 0, 2 * n)])
    for s in range(n):
        assert v[s] * 2.0**32 - 1.0 == words[2 * s] + words[2 * s + 1]
    # N = 1: v_s = u_s exactly, strictly inside (0, 1)
    spec1 = ScanSpec("linear", [np.arange(10.0)], np.zeros(1), np.ones(1), n, seed)
    v1 = zo.values(spec1, g)
    assert np.all(v1 > 0.0) and np.all(v1 < 1.0)
    assert [int(t) for t in (v1 * 2.0**32 - 0.5)] == words[:n]
