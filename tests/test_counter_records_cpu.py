"""Counter records (profiles/counter_records.txt) hold for the kernels now
built.  Each record names the id of the kernel it was taken on (a hash of its
gfx950 machine code and descriptor, read from libzmc.so): a kernel changed
after its counters were taken fails here, and bench.py then reports null for
that kernel's HBM traffic and VALU-counter fraction."""
import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402
from paper_1910_01965_amd import kernel_ids  # noqa: E402
from paper_1910_01965_amd import workloads as wl  # noqa: E402


@pytest.fixture(scope="module")
def ids():
    if not os.path.exists(kernel_ids.LIB):
        pytest.fail("libzmc.so is not built (run __graft_entry__.build())")
    return kernel_ids.kernel_ids()


def test_kernel_ids_are_read_from_the_library(ids):
    assert len(ids) > 500
    for name in (kernel_ids.GAUSS_F32_N3_POINT_MAJOR, kernel_ids.COSEXP_F32_N2_POINT_MAJOR,
                 kernel_ids.COSEXP_F64_N2_POINT_MAJOR):
        assert len(ids[name]) == 16
    # the float and double kernels of one family differ
    assert ids[kernel_ids.COSEXP_F32_N2_POINT_MAJOR] != ids[kernel_ids.COSEXP_F64_N2_POINT_MAJOR]


def test_every_record_was_taken_on_the_built_kernel(ids):
    records = bench.counter_records()
    assert records, "profiles/counter_records.txt holds no record"
    for r in records:
        assert r["kernel"] in ids, r["kernel"]
        assert ids[r["kernel"]] == r["kernel_id"], (
            f"{r['kernel']} changed since its counters were taken ({r['summary']}): "
            f"built {ids[r['kernel']]}, recorded {r['kernel_id']}")
        assert os.path.exists(os.path.join(ROOT, r["summary"])), r["summary"]


def test_records_cover_the_bench_kernels(ids):
    have = {(r["kernel"], r["workload"]) for r in bench.counter_records()}
    assert (kernel_ids.GAUSS_F32_N3_POINT_MAJOR, wl.gauss_2p().name) in have
    assert (kernel_ids.GAUSS_F64_N3_POINT_MAJOR, wl.gauss_2p().name) in have
    assert (kernel_ids.COSEXP_F32_N2_POINT_MAJOR, wl.cosexp_4p().name) in have


def test_a_reading_of_another_build_is_not_used(ids):
    rec = {"kernel_id": "0" * 16, "kernel": kernel_ids.GAUSS_F32_N3_POINT_MAJOR,
           "workload": "w", "fetch_bytes": 1.0, "write_bytes": 2.0, "valu_insts": 64.0,
           "valu_pairs": 0.0, "summary": "s"}
    assert bench.counter_record(rec["kernel"], "w", ids[rec["kernel"]], [rec]) is None
    good = dict(rec, kernel_id=ids[rec["kernel"]])
    assert bench.counter_record(rec["kernel"], "w", ids[rec["kernel"]], [good]) is good
