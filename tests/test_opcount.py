"""The algorithmic work per unit that bench.py prices its VALU roofline with
(lane-operations per test, draw and candidate) equals the VALU instruction
count of each decision's arithmetic in the gfx950 build of the library's own
device functions (tests/opcount_probe.hip, compiled here to assembly; each
unit kernel minus its twin with the same loads and stores)."""
import os
import re
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def valu_counts(tmp_path) -> dict:
    hipcc = os.environ.get("HIPCC") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc) and not shutil.which("hipcc"):
        pytest.skip("hipcc not found")
    out = os.path.join(tmp_path, "probe.s")
    subprocess.check_call([
        hipcc, "--offload-arch=gfx950", "-O3", "-std=c++17", "-ffp-contract=off", "-fno-fast-math",
        "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
        "-I", os.path.join(ROOT, "paper_1905_06706_amd", "csrc"), "-c", "--offload-device-only", "-S",
        os.path.join(ROOT, "tests", "opcount_probe.hip"), "-o", out], stderr=subprocess.DEVNULL)
    text = open(out).read()
    counts = {}
    for m in re.finditer(r"^((?:u|io)_\w+):[^\n]*\n(.*?)s_endpgm", text, re.S | re.M):
        ins = [ln.strip() for ln in m.group(2).splitlines()]
        counts[m.group(1)] = sum(1 for ln in ins if ln.startswith("v_"))
    return counts


def test_ops_per_unit_match_the_build(tmp_path):
    import bench
    c = valu_counts(str(tmp_path))
    unit = {k[2:]: c[k] - c["io_" + k[2:]] for k in c if k.startswith("u_")}
    philox = unit["philox"]          # one block = two type-I coins
    test_binom = unit["prob"] + philox / 2.0
    cand = unit["prob"]
    draw = unit["draw"]
    thresh = unit["thresh"]
    print(f"VALU per unit: {unit}; binomial test {test_binom}, draw {draw}, candidate {cand}, "
          f"threshold test {thresh}")
    for name, have, want in (("OPS_TEST_BINOM", bench.OPS_TEST_BINOM, test_binom),
                             ("OPS_DRAW", bench.OPS_DRAW, draw),
                             ("OPS_CAND", bench.OPS_CAND, cand),
                             ("OPS_TEST_T0", bench.OPS_TEST_T0, thresh)):
        assert abs(have - want) <= 0.1 * want, f"{name} = {have}, the build counts {want}"
