"""The C-ABI library loads and exports every entry point its header declares
(no compute calls: this runs without a GPU)."""
import ctypes
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    with open(os.path.join(ROOT, "include", "hipgirg.h")) as f:
        text = f.read()
    return sorted(set(re.findall(r"^\s*(?:girg_status|const char\*|int32_t)\s+(\w+)\s*\(", text, re.M)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for want in ("girg_generate", "girg_hrg", "girg_from_points", "girg_points", "girg_solve_c",
                 "hrg_solve_R", "girg_generate_batch", "girg_last_error"):
        assert want in names


def test_library_exports_every_declared_symbol():
    import paper_1905_06706_amd as hg
    if not os.path.exists(hg.LIB_PATH):
        from paper_1905_06706_amd import build
        build.build()
    lib = ctypes.CDLL(hg.LIB_PATH)
    for name in declared_functions():
        assert hasattr(lib, name), name
    assert set(declared_functions()) <= set(hg.EXPORTS)


def test_binding_fails_loudly_without_library(tmp_path, monkeypatch):
    import importlib
    import paper_1905_06706_amd as hg
    monkeypatch.setattr(hg, "LIB_PATH", str(tmp_path / "missing.so"))
    monkeypatch.setattr(hg, "_lib", None)
    try:
        hg.load()
    except ImportError:
        pass
    else:
        raise AssertionError("load() must raise without the built library")
    importlib.reload(hg)


def test_host_solvers_agree_with_oracle(orc):
    """girg_solve_c / girg_expected_degree / hrg_* run on the host side of the
    library (no device needed) and are independent implementations."""
    import numpy as np
    import paper_1905_06706_amd as hg
    from tests import synth
    w = synth.pareto_weights(20000, 2.4, 1)
    for d, T, deg in ((1, 0.0, 10.0), (2, 0.5, 16.0), (3, 0.8, 20.0)):
        c_lib = hg.solve_c(w, d, T, deg)
        c_orc = orc.solve_c(w, d, T, deg)
        assert abs(c_lib / c_orc - 1) < 1e-12
        assert abs(hg.expected_degree(w, d, T, c_orc) / orc.expected_avg_degree(w, d, T, c_orc) - 1) < 1e-12
    # heavy tails and low temperature: the closed form over all pairs and its
    # excess over E_R are both huge there; the sums must not cancel
    for n, d, beta, T, deg, seed in ((5689, 1, 2.283, 0.3, 15.8, 1008), (100000, 2, 2.1, 0.3, 30.0, 7),
                                     (20000, 1, 2.05, 0.2, 12.0, 3)):
        w = synth.pareto_weights(n, beta, seed)
        c_lib = hg.solve_c(w, d, T, deg)
        c_orc = orc.solve_c(w, d, T, deg)
        assert abs(c_lib / c_orc - 1) < 1e-12, (n, d, beta, T)
        assert abs(orc.expected_avg_degree(w, d, T, c_orc) / deg - 1) < 1e-13
    for T in (0.0, 0.5):
        a = hg.hrg_expected_degree(5000, 0.75, T, 16.0)
        b = orc.hrg_expected_avg_degree(5000, 0.75, T, 16.0)
        assert abs(a / b - 1) < 1e-6  # two independent quadratures
    R1 = hg.hrg_solve_R(4000, 0.75, 0.0, 10.0)
    R2 = orc.hrg_solve_R(4000, 0.75, 0.0, 10.0)
    assert abs(R1 - R2) < 1e-6
