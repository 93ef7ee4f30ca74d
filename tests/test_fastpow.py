"""pow_pos, the FP64 power of the pair probability (Eq. (1)), and log_pos, the
logarithm of a type-II draw's uniform (Sec. 3.2), built for the host from the
same header as the kernels and checked against the C library's pow and log:
relative errors within 2^-52 (6 + 2 |y log2 x|) and 3 2^-52 over 4·10^6
arguments each, capped probabilities within 1e-15 (far inside the 1e-12
near-boundary band), and exact results where the arithmetic fixes them."""
import json
import os
import subprocess

import pytest

from paper_1905_06706_amd.build import hipcc

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(os.path.dirname(HERE), "paper_1905_06706_amd", "csrc")


@pytest.fixture(scope="module")
def result(tmp_path_factory):
    exe = str(tmp_path_factory.mktemp("fastpow") / "fastpow_check")
    subprocess.run([hipcc(), "-x", "hip", "--offload-arch=gfx950", "-O2", "-ffp-contract=off",
                    "-fno-fast-math", "-I", CSRC, os.path.join(HERE, "fastpow_check.cpp"), "-o", exe],
                   check=True, capture_output=True)
    out = subprocess.run([exe], check=True, capture_output=True, text=True).stdout
    return json.loads(out)


def test_error_bound(result):
    assert result["cases"] > 3_000_000
    assert result["worst_rel_over_bound"] <= 1.0
    assert result["worst_abs_capped"] <= 1e-15


def test_log_error_bound(result):
    assert result["log_worst_rel_over_bound"] <= 1.0
    assert result["log1"] == 0.0
    assert result["log2"] == 0.6931471805599453


def test_exact_cases(result):
    assert result["p2_10"] == 1024.0
    assert result["p05_3"] == 0.125
    assert result["p1_7"] == 1.0
    assert abs(result["px_1"] - 0.3) <= 2 * 2.0 ** -54
    assert result["p0"] == 0.0
    assert result["pinf_is_inf"] == 1
    assert result["tiny"] == 0.0
