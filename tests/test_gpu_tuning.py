"""Launch-shape tuning on the GPU: the number of workgroups of the
persistent sampling passes changes no edge and no position (1 to 2048
workgroups give one edge array), and the autotuners store a candidate
without changing any result."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def hg():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1905_06706_amd as hg
    hg.load()
    hg.tuning_reset()
    yield hg
    hg.tuning_reset()


CASES = [
    dict(n=2**16, d=2, beta=2.7, T=0.5, avg_deg=16.0, seed=21),   # split and segmented passes
    dict(n=40000, d=1, beta=2.5, T=0.0, avg_deg=10.0, seed=22),   # threshold
    dict(n=30000, d=3, beta=2.3, T=0.8, avg_deg=20.0, seed=23, precision=1),
]


@pytest.mark.parametrize("case", CASES, ids=["d2T05", "d1T0", "d3mixed"])
def test_grid_size_changes_nothing(hg, case):
    ref = hg.generate(**case)
    p = hg.make_params(case["n"], case["d"], case["beta"], case["T"], case["avg_deg"], 0.0, case["seed"],
                       case.get("precision", 0))
    try:
        for blocks in (1, 3, 37, 2048):
            print(f"[tuning] {case} blocks={blocks}", flush=True)
            hg.tuning_set(p, blocks)
            assert hg.tuning_get(p)[0] == blocks
            r = hg.generate(**case)
            assert np.array_equal(r.edges.cpu().numpy(), ref.edges.cpu().numpy()), blocks
            for k in ("tests", "draws", "candidates", "type1_edges", "type2_edges", "split_items", "heavy_items"):
                assert r.info[k] == ref.info[k], (blocks, k)
    finally:
        hg.tuning_reset()


def test_grid_size_hrg(hg):
    ref = hg.hrg(30000, 0.75, T=0.5, avg_deg=10.0, seed=24)
    p = hg.make_params(30000, 1, 0.0, 0.5, 10.0, model=1, alpha=0.75)
    try:
        hg.tuning_set(p, 5)
        r = hg.hrg(30000, 0.75, T=0.5, avg_deg=10.0, seed=24)
        assert np.array_equal(r.edges.cpu().numpy(), ref.edges.cpu().numpy())
    finally:
        hg.tuning_reset()


def test_autotune_single(hg):
    case = dict(n=2**15, d=2, beta=2.7, T=0.5, avg_deg=16.0, seed=25)
    ref = hg.generate(**case)
    p = hg.make_params(case["n"], case["d"], case["beta"], case["T"], case["avg_deg"], 0.0, case["seed"])
    try:
        b = hg.autotune(p, reps=2)
        assert b in (256, 512, 768, 1024, 1536, 2048)
        assert hg.tuning_get(p)[0] == b
        r = hg.generate(**case)
        assert np.array_equal(r.edges.cpu().numpy(), ref.edges.cpu().numpy())
    finally:
        hg.tuning_reset()


def test_autotune_batch(hg):
    rng = np.random.default_rng(31)
    P = [hg.make_params(int(rng.integers(500, 6000)), 1 + b % 2, float(rng.uniform(2.1, 3.0)),
                        [0.0, 0.3, 0.9][b % 3], float(rng.uniform(8, 24)), 0.0, 900 + b) for b in range(10)]
    e0, o0, _ = hg.generate_batch(P)
    try:
        b, w = hg.autotune_batch(P, reps=1)
        assert b in (128, 256, 512, 768, 1024) and w in (8, 16)
        assert hg.tuning_get(P[0], batch=True) == (b, w)
        e1, o1, _ = hg.generate_batch(P)
        assert o0 == o1
        assert np.array_equal(e0.cpu().numpy(), e1.cpu().numpy())
    finally:
        hg.tuning_reset()
