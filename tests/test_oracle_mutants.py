"""The pins catch plausible mistakes: each case plants one mistake in a copy of
the oracle's source (a wrong index, a dropped term or factor, an off-by-one,
a reused random stream), builds it, and runs a pin against it; the pin must
fail.  The oracle itself is never changed.  (The same pins pass on the
unchanged oracle in the other test modules.)"""
import os

import pytest

import oracle
from tests import test_oracle_degree as deg
from tests import test_oracle_primitives as prim
from tests import test_oracle_sampler as smp
from tests import test_oracle_batched as bat
from tests import test_oracle_segments as seg

SRC = os.path.join(os.path.dirname(oracle.__file__), "oracle.c")


def pin_segments(orc):
    seg.test_segmented_items_chi_square_and_independence(orc, 1, 0.5)


def pin_type1_chi2(orc):
    smp.test_binomial_girg_chi_square(orc, 2, 14, 0.3, 2)


def pin_variance(orc):
    smp.test_binomial_edge_count_variance(orc, -2)


def pin_threshold(orc):
    smp.test_threshold_girg_equals_bruteforce(orc, 2, 2000, 2.1, 9, True)


def pin_hrg_threshold(orc):
    smp.test_threshold_hrg_equals_literal_formula(orc)


def pin_expected_degree(orc):
    deg.test_expected_degree_matches_pairwise_integral(orc, 2, 0.3)


def pin_morton(orc):
    prim.test_morton_paper_example(orc)


def pin_coverage(orc):
    smp.test_coverage_every_pair_exactly_once(orc, 2, 2, -1)


def pin_batched_chi2(orc):
    bat.test_batched_chi_square(orc, 2, 16, 0.4, 4)


def pin_batched_coverage(orc):
    bat.test_batched_coverage_every_pair_exactly_once(orc, 2)


# (name, text in oracle.c, its replacement, the pin that must fail)
MUTANTS = [
    ("segment start skips a candidate", "uint64_t k = s * G, kend",
     "uint64_t k = s * G + (s == 1), kend", pin_segments),
    ("segment end one short", "(s + 1) * G < N ? (s + 1) * G : N;",
     "(s + 1) * G < N ? (s + 1) * G - 1 : N;", pin_segments),
    ("segments overlap by one", "(s + 1) * G < N ? (s + 1) * G : N;",
     "(s + 1) * G < N ? (s + 1) * G + 1 : N;", pin_segments),
    ("one jump sequence for every segment", "word3(l, i, j, KIND_TYPE2, (uint32_t)s)",
     "word3(l, i, j, KIND_TYPE2, 0u)", pin_segments),
    ("acceptance without the bound", "if (Acc * pbar < prob) emit(R, u, v, 1);",
     "if (Acc < prob) emit(R, u, v, 1);", pin_segments),
    ("skip rate of half the bound", "double Lg = log1p(-pbar);",
     "double Lg = log1p(-0.5 * pbar);", pin_segments),
    ("cell distance one cell too far", "double dist = ldexp((double)g, -l);",
     "double dist = ldexp((double)g + 1.0, -l);", pin_segments),
    ("type-I pairs share a coin word", "int h = (int)(k & 1);", "int h = 0;", pin_variance),
    ("probability exponent T instead of 1/T", "pow((wu * wv / R->W) / rd, 1.0 / R->p.T)",
     "pow((wu * wv / R->W) / rd, R->p.T)", pin_type1_chi2),
    ("no wrap-around in the torus distance",
     "double m = delta < 1.0 - delta ? delta : 1.0 - delta;", "double m = delta;", pin_threshold),
    ("threshold comparison level one too deep",
     "while (l < Dcap && ldexp(1.0, -(l + 1)) >= tmax) l++;",
     "while (l < Dcap && ldexp(1.0, -(l + 1)) >= 0.5 * tmax) l++;", pin_threshold),
    ("HRG distance without the factor 2",
     "return cosh(ru - rv) + 2.0 * sinh(ru) * sinh(rv) * s * s;",
     "return cosh(ru - rv) + sinh(ru) * sinh(rv) * s * s;", pin_hrg_threshold),
    ("expected degree: 1 - T in the numerator", "cT * ldexp(1.0, d) / (1.0 - T)",
     "cT * ldexp(1.0, d) * (1.0 - T)", pin_expected_degree),
    ("Morton code with the dimensions transposed", "int pos = b * d + (d - 1 - k);",
     "int pos = b * d + k;", pin_morton),
    ("neighbour pairs miss the own-cell layer pairs", "if (A == B && j < i) continue;",
     "if (A == B && j <= i) continue;", pin_coverage),
    ("sequences: acceptance without the bound", "if (pbar * Acc < puv) emit(R, u, v, 1);",
     "if (Acc < puv) emit(R, u, v, 1);", pin_batched_chi2),
    ("sequences: skip rate of half the bound", "double lg1 = log1p(-pbar);",
     "double lg1 = log1p(-0.5 * pbar);", pin_batched_chi2),
    ("sequences: the last cell pair never sampled", "for (int k = 0; k < nit; k++) total +=",
     "for (int k = 0; k + 1 < nit; k++) total +=", pin_batched_coverage),
]


@pytest.mark.parametrize("name,old,new,pin", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_pin_catches_planted_mistake(orc, tmp_path, name, old, new, pin):
    with open(SRC) as fh:
        text = fh.read()
    assert text.count(old) == 1, f"mutation site not unique: {old!r}"
    lib = oracle.build_variant(text.replace(old, new), str(tmp_path / "liboracle_variant.so"))
    with oracle.use_library(lib):
        with pytest.raises(AssertionError):
            pin(oracle)
