"""Planted mistakes: every plausible slip in the oracle must fail a pin.

Each mutant is a copy of oracle/zmc_oracle.c with one textual change (a
dropped term, a wrong sign or index, a transposed operand), compiled on the
CPU into a temporary library.  The pins of test_oracle_philox,
test_oracle_estimator and test_oracle_closed_forms are then run against it;
at least one must fail.  This shows that the pins constrain the oracle, not
only that the oracle passes them.
"""
import os

import pytest

from oracle import build as obuild
from oracle import oracle as zo

import test_oracle_closed_forms as tcf
import test_oracle_estimator as tes
import test_oracle_philox as tph

SRC = obuild.SRC

MUTANTS = [
    ("philox multipliers swapped", "PHILOX_M0 * (uint64_t)r0", "PHILOX_M1 * (uint64_t)r0"),
    ("philox key not bumped", "k0 += PHILOX_W0;", "k0 += 0u;"),
    ("philox key not mixed in", "hi1 ^ r1 ^ k0", "hi1 ^ r1"),
    ("philox output lanes rotated", "out[0] = r0; out[1] = r1;", "out[0] = r1; out[1] = r0;"),
    ("word order transposed", "uint64_t w = s * (uint64_t)spec->N + (uint64_t)k;",
     "uint64_t w = (uint64_t)k * spec->samples + s;"),
    ("uniform without half offset", "((double)r + 0.5) * 0x1p-32", "((double)r) * 0x1p-32"),
    ("map drops the lower edge", "fma(h, u, spec->lo[k])", "fma(h, u, 0.0)"),
    ("gauss drops its coefficient", "double c = (k < M) ? x[k] : 1.0;", "double c = 1.0;"),
    ("gauss coefficient transposed", "double c = (k < M) ? x[k] : 1.0;",
     "double c = (k < M) ? x[M - 1 - k] : 1.0;"),
    ("cosexp exponent sign", "exp(-(x[2] * x[2]) * y[0] * y[1])", "exp((x[2] * x[2]) * y[0] * y[1])"),
    ("cosexp drops x4", "* y[0] * y[1]) + x[3];", "* y[0] * y[1]);"),
    ("cosexp phase operands transposed", "x[0] * y[0] + x[1] * y[1]", "x[0] * y[1] + x[1] * y[0]"),
    ("sin_sum drops the parameters", "return sin(sx + sy);", "return sin(sy);"),
    ("grid decoded first-axis-fastest", "for (l = spec->M - 1; l >= 0; --l) {",
     "for (l = 0; l < spec->M; ++l) {"),
    ("no Bessel correction", "((double)n * (double)(n - 1))", "((double)n * (double)n)"),
    ("mean over n - 1", "mu = nsum_value(&sum) / (double)n;", "mu = nsum_value(&sum) / (double)(n - 1);"),
    ("volume from upper edges", "V *= spec->hi[k] - spec->lo[k];", "V *= spec->hi[k];"),
]

_ROCRAND = {}


def _word_order_pin():
    # the exact word-stream pin needs the rocRAND cross-check generator
    if "exe" not in _ROCRAND:
        import tempfile
        _ROCRAND["exe"] = tph.build_rocrand_exe(tempfile.mkdtemp(prefix="zmc_rocrand_"))
    if _ROCRAND["exe"] is not None:
        tph.test_sample_coordinates_follow_word_order(_ROCRAND["exe"])


PINS = [
    tph.test_published_known_answers,
    _word_order_pin,
    tcf.test_gauss_general_box,
    tes.test_const_family_is_exact_volume,
    tes.test_two_samples_special_case,
    tes.test_grid_decoding_is_c_order,
    tcf.test_sin_sum_plain_shape_coverage,
    tcf.test_gauss_two_parameter_coverage,
    tcf.test_cosexp_special_cases_of_quadrature,
    tcf.test_cosexp_coverage_against_quadrature,
    tcf.test_linear_coverage,
    tcf.test_sin_sum_paper_box_coverage,
]


def _fails_a_pin():
    for pin in PINS:
        try:
            pin()
        except (AssertionError, ValueError):
            return pin.__name__
    return None


@pytest.mark.parametrize("name,old,new", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_planted_mistake_is_caught(name, old, new, tmp_path, monkeypatch):
    src = open(SRC).read()
    assert src.count(old) == 1, f"mutation site not unique: {old}"
    mutant = tmp_path / "zmc_oracle_mutant.c"
    mutant.write_text(src.replace(old, new))
    lib = obuild.build(out=str(tmp_path / "libmutant.so"), src=str(mutant), extra=("-w",))
    monkeypatch.setattr(zo, "_lib", zo.load(lib))
    caught = _fails_a_pin()
    assert caught is not None, f"no pin fails for mutant '{name}'"


def test_unmutated_oracle_passes_every_pin():
    assert _fails_a_pin() is None
    assert os.path.exists(obuild.LIB)
