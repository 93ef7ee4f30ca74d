"""GPU parity at the benchmark sizes, through the same entry points the
benchmark times (girg_generate, girg_hrg): whole edge sets where the oracle
finishes in seconds, a cell-pair sample of the edge set where it does not,
and the mixed-precision path against the FP64 path bit for bit."""
import numpy as np
import pytest

from tests.parity import compare, level3_sample

pytestmark = pytest.mark.gpu


def gpu_points(hg, n, d, beta, seed):
    """The GPU's points (the kernel girg_generate runs), on the host as the
    oracle takes them: w (n,), x (n, d)."""
    w, x = hg.points(n, d, beta, seed=seed)
    return w.cpu().numpy(), np.ascontiguousarray(x.cpu().numpy().T)


@pytest.fixture(scope="module")
def hg():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1905_06706_amd as hg
    hg.load()
    return hg


def test_fullsize_girg_d2_n2p20(hg, orc):
    """GIRG d = 2, n = 2^20, beta = 2.7, T = 0.5, average degree 16, seed 2:
    the whole edge set."""
    n, d, beta, T, deg, seed = 2**20, 2, 2.7, 0.5, 16.0, 2
    print(f"[fullsize] girg n={n} d={d} T={T}", flush=True)
    res = hg.generate(n, d=d, beta=beta, T=T, avg_deg=deg, seed=seed)
    w, x = gpu_points(hg, n, d, beta, seed)
    assert res.info["c"] == pytest.approx(orc.solve_c(w, d, T, deg), rel=1e-12)
    run = orc.run(w, x, T=T, c=res.info["c"], seed=seed, keep=True)
    rep = compare(res.edges.cpu().numpy().view(np.uint32), run, info=res.info)
    assert rep["gpu"] > 7 * n
    assert res.info["tests"] == run.stats["tests"]
    assert res.info["draws"] == run.stats["draws"]
    assert res.info["candidates"] == run.stats["candidates"]


def test_fullsize_hrg_n2p20(hg, orc):
    """HRG n = 2^20, alpha = 0.75, T = 0.5, average degree 10 (R solved),
    seed 3: the whole edge set."""
    n, alpha, T, deg, seed = 2**20, 0.75, 0.5, 10.0, 3
    print(f"[fullsize] hrg n={n} alpha={alpha} T={T}", flush=True)
    res = hg.hrg(n, alpha, T=T, avg_deg=deg, seed=seed)
    R = orc.hrg_solve_R(n, alpha, T, deg)
    assert res.info["R"] == pytest.approx(R, rel=1e-6)
    # the sampler's R (its own quadrature) decides the graph: run the oracle on it
    R = res.info["R"]
    r, x = hg.points(n, model=1, alpha=alpha, R=R, seed=seed)
    run = orc.run(r.cpu().numpy(), x.cpu().numpy().T, T=T, model=1, R=R, alpha=alpha, seed=seed, keep=True)
    rep = compare(res.edges.cpu().numpy().view(np.uint32), run, info=res.info)
    assert rep["gpu"] > 4 * n


def test_fullsize_girg_d3_n1e7_sampled(hg, orc):
    """GIRG d = 3, n = 10^7, beta = 2.3, T = 0.8, average degree 20, seed 4,
    the FP32 filter with FP64 recheck (the benchmark's reported leg): every
    item above level 3 and 1/512 of the level-3 subtrees."""
    import torch
    n, d, beta, T, deg, seed = 10**7, 3, 2.3, 0.8, 20.0, 4
    print(f"[fullsize] girg n={n} d={d} T={T} sampled", flush=True)
    res = hg.generate(n, d=d, beta=beta, T=T, avg_deg=deg, seed=seed, precision=1)
    wd, xd = hg.points(n, d, beta, seed=seed)
    w, x = wd.cpu().numpy(), np.ascontiguousarray(xd.cpu().numpy().T)
    assert res.info["c"] == pytest.approx(orc.solve_c(w, d, T, deg), rel=1e-12)
    run = orc.run(w, x, T=T, c=res.info["c"], seed=seed, keep=True, filter_level=3, filter_mod=512,
                  filter_rem=0)
    sub = level3_sample(res.edges, xd, run, 512)
    rep = compare(sub.cpu().numpy().view(np.uint32), run)
    assert rep["oracle"] > 10**6
    del xd, sub


def test_fullsize_mixed_equals_fp64_d3_n1e7(hg):
    """The FP32 filter with FP64 recheck returns the FP64 path's edge array
    bit for bit at n = 10^7, d = 3, T = 0.8."""
    import torch
    kw = dict(d=3, beta=2.3, T=0.8, avg_deg=20.0, seed=4)
    print("[fullsize] mixed vs fp64 n=1e7 d=3", flush=True)
    a = hg.generate(10**7, precision=0, **kw)
    b = hg.generate(10**7, precision=1, **kw)
    assert a.edges.shape == b.edges.shape
    assert torch.equal(a.edges, b.edges)
    assert a.info["rechecks"] == 0
    assert 0 < b.info["rechecks"] < b.info["tests"] + b.info["draws"] + b.info["candidates"]
    for k in ("tests", "draws", "candidates", "type1_edges", "type2_edges"):
        assert a.info[k] == b.info[k], k


def test_fullsize_girg_d3_n1e7_whole(hg):
    """GIRG d = 3, n = 10^7, beta = 2.3, T = 0.8, average degree 20, seed 4,
    the FP32 filter with FP64 recheck: the whole edge set (about 10^8 edges)
    against the oracle on the GPU's points and c, the oracle's run split over
    host processes (level-3 subtrees plus the levels above)."""
    from tests.oracle_pool import run_whole, workers
    from tests.parity import compare_large
    n, d, beta, T, deg, seed = 10**7, 3, 2.3, 0.8, 20.0, 4
    print(f"[fullsize] girg n={n} d={d} T={T} whole, {workers()} oracle processes", flush=True)
    res = hg.generate(n, d=d, beta=beta, T=T, avg_deg=deg, seed=seed, precision=1)
    ge = res.edges.cpu().numpy().view(np.uint32)
    w, x = gpu_points(hg, n, d, beta, seed)
    run = run_whole(w, x, level=3, nparts=32, T=T, c=res.info["c"], seed=seed)
    print(f"[fullsize] oracle: {len(run.edges)} edges, {len(run.near)} near, {len(run.ties)} tie items",
          flush=True)
    rep = compare_large(ge, run, info=res.info)
    print(f"[fullsize] {rep}", flush=True)
    assert rep["gpu"] > 5 * n
    for k in ("tests", "draws", "candidates"):
        assert res.info[k] == run.stats[k], k


def test_fullsize_girg_d3_n1e7_batched_sampled(hg, orc):
    """The same graph with batched type-II sequences (type2_batch = 1), the
    FP32 filter with FP64 recheck: every item above level 3 and the sequences
    of 1/512 of the level-3 subtrees (by the source cell's ancestor) against
    the oracle's batched run on the GPU's points and c."""
    n, d, beta, T, deg, seed = 10**7, 3, 2.3, 0.8, 20.0, 4
    print(f"[fullsize] girg n={n} d={d} T={T} batched sampled", flush=True)
    res = hg.generate(n, d=d, beta=beta, T=T, avg_deg=deg, seed=seed, precision=1, type2_batch=1)
    wd, xd = hg.points(n, d, beta, seed=seed)
    w, x = wd.cpu().numpy(), np.ascontiguousarray(xd.cpu().numpy().T)
    run = orc.run(w, x, T=T, c=res.info["c"], seed=seed, keep=True, filter_level=3, filter_mod=512,
                  filter_rem=0, batch_type2=True)
    sub = level3_sample(res.edges, xd, run, 512, batched=True)
    rep = compare(sub.cpu().numpy().view(np.uint32), run)
    assert rep["oracle"] > 10**6
    del xd, sub
