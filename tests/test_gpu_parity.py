"""GPU parity: the HIP path (through the C ABI) against the oracle on the same
seeded inputs.  Edge sets must match except for the pairs the oracle logs as
near the decision boundary; indices, layers and level tables bit-exactly."""
import numpy as np
import pytest

from tests import synth
from tests.parity import compare

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def hg():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1905_06706_amd as hg
    hg.load()
    return hg


def dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def run_both(hg, orc, w, x, *, T, c, seed, model=0, R=0.0, alpha=0.0, **kw):
    print(f"[parity] n={len(w)} d={x.shape[1]} T={T} c={c} seed={seed} model={model} {kw}", flush=True)
    res = hg.from_points(dev(w), dev(x.T), T=T, c=c, seed=seed, model=model, R=R, alpha=alpha, **kw)
    ge = res.edges.cpu().numpy().view(np.uint32)
    kw.pop("precision", None)  # the oracle decides in FP64 only
    if kw.pop("type2_batch", 0):
        kw["batch_type2"] = True
    run = orc.run(w, x, T=T, c=c, seed=seed, model=model, R=R, alpha=alpha, keep=True, **kw)
    return ge, res.info, run


def test_points_match_oracle(hg, orc):
    for d in (1, 2, 3, 4):
        w, x = hg.points(20000, d, 2.3, seed=7)
        ow, ox = orc.points_girg(20000, d, 2.3, 7)
        assert np.array_equal(x.cpu().numpy(), ox.T)  # positions: pure integer arithmetic
        rel = np.abs(w.cpu().numpy() - ow) / ow
        assert rel.max() <= 4.5e-16                     # weights: pow within 2 ulp
    r, x = hg.points(20000, model=1, alpha=0.75, R=20.0, seed=3)
    orr, ox = orc.points_hrg(20000, 0.75, 20.0, 3)
    assert np.array_equal(x.cpu().numpy()[0], ox[:, 0])
    assert np.max(np.abs(r.cpu().numpy() - orr)) <= 1e-13


@pytest.mark.parametrize("d,n,beta,seed", [(1, 10000, 2.5, 1), (2, 20000, 2.7, 2), (3, 20000, 2.3, 4), (4, 8000, 2.6, 5)])
def test_threshold_from_points(hg, orc, d, n, beta, seed):
    w = synth.pareto_weights(n, beta, seed)
    x = synth.positions(n, d, seed)
    c = orc.solve_c(w, d, 0.0, 10.0)
    ge, info, run = run_both(hg, orc, w, x, T=0.0, c=c, seed=seed)
    rep = compare(ge, run, info=info)
    assert info["L"] == run.stats["L"] and info["D"] == run.stats["D"]
    # W: the GPU's sum (double-double) and the oracle's plain ascending sum
    # differ at most by the latter's rounding, (n - 1) u W
    assert abs(info["W"] - run.stats["W"]) <= (n - 1) * 2.0**-53 * run.stats["W"]
    assert rep["gpu"] > n


@pytest.mark.parametrize("d,n,T,seed", [(1, 8000, 0.5, 3), (2, 12000, 0.5, 2), (3, 6000, 0.8, 4), (2, 6000, 0.3, 9),
                                        (1, 5000, 0.9, 11), (4, 3000, 0.6, 12), (4, 2500, 0.2, 13)])
def test_binomial_from_points(hg, orc, d, n, T, seed):
    w = synth.pareto_weights(n, 2.5, seed)
    x = synth.positions(n, d, seed)
    c = orc.solve_c(w, d, T, 12.0)
    ge, info, run = run_both(hg, orc, w, x, T=T, c=c, seed=seed)
    rep = compare(ge, run, info=info)
    assert info["tests"] == run.stats["tests"]
    assert info["draws"] == run.stats["draws"]
    assert info["candidates"] == run.stats["candidates"]
    assert info["type2_edges"] == run.stats["type2_edges"]


@pytest.mark.parametrize("bias,depth", [(2, -1), (-2, -1), (0, 1), (0, 0), (3, 4)])
def test_binomial_level_knobs(hg, orc, bias, depth):
    n, d, T = 3000, 2, 0.5
    w = synth.pareto_weights(n, 2.2, 5)
    x = synth.clustered_positions(n, d, 5)
    c = orc.solve_c(w, d, T, 14.0)
    ge, info, run = run_both(hg, orc, w, x, T=T, c=c, seed=5, cl_bias=bias, max_depth=depth)
    compare(ge, run, info=info)


def test_heavy_items_split_into_segments(hg, orc):
    # coarse levels for low weights: type-II items with many expected candidates
    n, d, T = 20000, 1, 0.9
    w = synth.pareto_weights(n, 2.8, 6)
    x = synth.positions(n, d, 6)
    c = orc.solve_c(w, d, T, 20.0)
    ge, info, run = run_both(hg, orc, w, x, T=T, c=c, seed=6)
    assert info["heavy_items"] > 0
    compare(ge, run, info=info)
    assert info["draws"] == run.stats["draws"]


@pytest.mark.parametrize("T", [0.0, 0.5, 0.9])
def test_hrg_from_points(hg, orc, T):
    n, alpha = 20000, 0.75
    R = orc.hrg_solve_R(n, alpha, T, 10.0)
    r = synth.hrg_radii(n, alpha, R, 3)
    x = synth.positions(n, 1, 3)
    ge, info, run = run_both(hg, orc, r, x, T=T, c=0.0, seed=3, model=1, R=R, alpha=alpha)
    compare(ge, run, info=info)


def gpu_points(hg, n, d, beta, seed):
    """The GPU's points (the same kernel girg_generate runs), on the host as
    the oracle takes them: w (n,), x (n, d)."""
    w, x = hg.points(n, d, beta, seed=seed)
    return w.cpu().numpy(), np.ascontiguousarray(x.cpu().numpy().T)


def test_generate_end_to_end_config1(hg, orc):
    """n = 10^4, d = 1, beta = 2.5, T = 0, average degree 10, seed 1: the GPU
    generates points, solves c and samples; the oracle samples the GPU's
    points with the GPU's c (its own c solve agrees to 1e-12); edge sets agree."""
    res = hg.generate(10**4, d=1, beta=2.5, T=0.0, avg_deg=10.0, seed=1)
    ge = res.edges.cpu().numpy().view(np.uint32)
    w, x = gpu_points(hg, 10**4, 1, 2.5, 1)
    assert res.info["c"] == pytest.approx(orc.solve_c(w, 1, 0.0, 10.0), rel=1e-12)
    run = orc.run(w, x, T=0.0, c=res.info["c"], seed=1, keep=True)
    compare(ge, run, info=res.info)


def test_generate_end_to_end_binomial(hg, orc):
    n, d, beta, T, deg, seed = 2**15, 2, 2.7, 0.5, 16.0, 2
    res = hg.generate(n, d=d, beta=beta, T=T, avg_deg=deg, seed=seed)
    ge = res.edges.cpu().numpy().view(np.uint32)
    w, x = gpu_points(hg, n, d, beta, seed)
    assert res.info["c"] == pytest.approx(orc.solve_c(w, d, T, deg), rel=1e-12)
    run = orc.run(w, x, T=T, c=res.info["c"], seed=seed, keep=True)
    compare(ge, run, info=res.info)


def test_deterministic_output(hg):
    a = hg.generate(50000, d=2, beta=2.5, T=0.5, avg_deg=12.0, seed=9).edges.cpu().numpy()
    b = hg.generate(50000, d=2, beta=2.5, T=0.5, avg_deg=12.0, seed=9).edges.cpu().numpy()
    assert np.array_equal(a, b)


def test_overflow_reports_needed_capacity(hg):
    import ctypes
    import torch
    L = hg.load()
    p = hg.make_params(20000, 2, 2.5, 0.5, 10.0, 0.0, 3)
    buf = torch.empty((10, 2), dtype=torch.int32, device="cuda")
    m = ctypes.c_uint64(0)
    st = L.girg_generate(ctypes.byref(p), ctypes.c_void_p(buf.data_ptr()), 10, ctypes.byref(m), None,
                         ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert st == hg.GIRG_EOVERFLOW
    full = hg.generate(20000, d=2, beta=2.5, T=0.5, avg_deg=10.0, seed=3)
    assert m.value == full.edges.shape[0]


def test_invalid_parameters(hg):
    with pytest.raises(hg.GirgError):
        hg.generate(1000, d=5, beta=2.5, avg_deg=10)
    with pytest.raises(hg.GirgError):
        hg.generate(1000, d=2, beta=1.9, avg_deg=10)
    with pytest.raises(hg.GirgError):
        hg.generate(1000, d=2, beta=2.5, T=1.0, avg_deg=10)
    with pytest.raises(hg.GirgError):
        hg.generate(1000, d=2, beta=2.5, avg_deg=10, c=1.0)


def test_empty_and_tiny_graphs(hg, orc):
    for n in (2, 3, 17):
        w = synth.pareto_weights(n, 2.5, n)
        x = synth.positions(n, 2, n)
        ge, info, run = run_both(hg, orc, w, x, T=0.5, c=0.05, seed=1)
        compare(ge, run, info=info)
    # a graph with no edges at all
    w = np.ones(64)
    x = synth.positions(64, 3, 1)
    ge, info, run = run_both(hg, orc, w, x, T=0.0, c=1e-9, seed=1)
    assert len(ge) == 0 and len(run.edges) == 0


@pytest.mark.parametrize("T,d", [(0.0, 2), (0.5, 2), (0.0, 3), (0.8, 3)])
def test_torus_seam(hg, orc, T, d):
    """Points within 2^-4 of the seam 0 = 1 in every coordinate (c scaled down
    by 8 for the density): pairs on the two sides are near only through the
    wrap-around of the torus distance, and their cells are neighbours (type
    I) or distant (type II) only modulo 2^level."""
    n = 4000
    w = synth.pareto_weights(n, 2.5, 17)
    x = synth.seam_positions(n, d, 17, width=2.0**-4)
    c = orc.solve_c(w, d, T, 10.0) / 8.0
    ge, info, run = run_both(hg, orc, w, x, T=T, c=c, seed=17)
    compare(ge, run, info=info)
    assert info["tests"] == run.stats["tests"] and info["draws"] == run.stats["draws"]
    # a share of the edges joins the two sides of the seam (7-53 % here)
    e = ge.astype(np.int64)
    cross = np.any((x[e[:, 0]] < 0.5) != (x[e[:, 1]] < 0.5), axis=1)
    assert cross.mean() > 0.05
    if T > 0.0:
        assert run.stats["type2_items"] > 1000


@pytest.mark.parametrize("T,d", [(0.0, 2), (0.5, 2), (0.5, 3), (0.9, 1)])
def test_degenerate_one_point_one_layer(hg, orc, T, d):
    """Every vertex at one position and of one weight: one layer, every pair in
    one cell at every level (a single triangular type-I item per level pair,
    split into pieces), distance 0 so p_uv = 1: the complete graph, by the
    oracle and by the closed form n (n - 1) / 2."""
    n = 1500
    w = np.full(n, 3.0)
    x = np.full((n, d), 0.3125)
    ge, info, run = run_both(hg, orc, w, x, T=T, c=0.5, seed=7)
    compare(ge, run, info=info)
    assert len(ge) == n * (n - 1) // 2
    assert info["split_items"] > 0
    pairs = np.sort(ge.astype(np.int64), axis=1)
    assert len(np.unique(pairs[:, 0] * n + pairs[:, 1])) == n * (n - 1) // 2


@pytest.mark.parametrize("d,n,beta,T,seed", [(1, 2**16, 2.5, 0.5, 21), (2, 2**17, 2.7, 0.5, 22),
                                             (3, 2**17, 2.3, 0.8, 23), (4, 2**15, 2.6, 0.3, 24),
                                             (2, 2**16, 2.1, 0.9, 25)])
def test_mixed_precision_equals_fp64(hg, d, n, beta, T, seed):
    """precision = 1 (FP32 filter, FP64 recheck near the boundary) gives the
    FP64 edge array bit for bit, and reports its rechecks."""
    print(f"[mixed] d={d} n={n} beta={beta} T={T} seed={seed}", flush=True)
    kw = dict(d=d, beta=beta, T=T, avg_deg=16.0, seed=seed)
    a = hg.generate(n, precision=0, **kw)
    b = hg.generate(n, precision=1, **kw)
    assert np.array_equal(a.edges.cpu().numpy(), b.edges.cpu().numpy())
    assert a.info["rechecks"] == 0 and b.info["rechecks"] > 0
    for k in ("tests", "draws", "candidates", "type1_edges", "type2_edges"):
        assert a.info[k] == b.info[k], k


@pytest.mark.parametrize("d,T,seed", [(2, 0.5, 31), (3, 0.8, 32), (1, 0.2, 33)])
def test_mixed_precision_from_points(hg, orc, d, T, seed):
    """Mixed precision on clustered positions (many small distances) and
    heavy-tailed weights against the oracle."""
    n = 12000
    w = synth.pareto_weights(n, 2.1, seed)
    x = synth.clustered_positions(n, d, seed)
    c = orc.solve_c(w, d, T, 14.0)
    ge, info, run = run_both(hg, orc, w, x, T=T, c=c, seed=seed, precision=1)
    compare(ge, run, info=info)
    assert info["rechecks"] > 0
    assert info["draws"] == run.stats["draws"]
    assert info["candidates"] == run.stats["candidates"]


def test_mixed_precision_ignored_where_undefined(hg):
    """Threshold graphs and HRGs have no FP32 filter: precision = 1 runs the
    FP64 decisions and reports no rechecks."""
    a = hg.generate(20000, d=2, beta=2.5, T=0.0, avg_deg=10.0, seed=3, precision=0)
    b = hg.generate(20000, d=2, beta=2.5, T=0.0, avg_deg=10.0, seed=3, precision=1)
    assert np.array_equal(a.edges.cpu().numpy(), b.edges.cpu().numpy())
    assert b.info["rechecks"] == 0


@pytest.mark.parametrize("n,d,beta,T,deg,seed", [(2**16, 3, 2.1, 0.8, 30.0, 41), (2**17, 1, 2.05, 0.3, 40.0, 42),
                                                 (2**15, 2, 2.2, 0.0, 60.0, 43)])
def test_c_solve_with_a_large_heavy_tail(hg, orc, n, d, beta, T, deg, seed):
    """Heavy tails whose E_R reaches far below the heaviest layers: the device
    c solve must grow its tail and still agree with the oracle."""
    res = hg.generate(n, d=d, beta=beta, T=T, avg_deg=deg, seed=seed)
    w, x = gpu_points(hg, n, d, beta, seed)
    assert res.info["c"] == pytest.approx(orc.solve_c(w, d, T, deg), rel=1e-12)
    run = orc.run(w, x, T=T, c=res.info["c"], seed=seed, keep=True)
    compare(res.edges.cpu().numpy().view(np.uint32), run, info=res.info)


@pytest.mark.parametrize("d,n,T,seed,prec,bias", [(2, 12000, 0.5, 2, 0, 0), (3, 9000, 0.8, 4, 0, 0),
                                                  (3, 9000, 0.8, 4, 1, 0), (2, 6000, 0.3, 9, 1, 2),
                                                  (3, 4000, 0.6, 12, 0, 2), (2, 20000, 0.9, 13, 0, -1)])
def test_batched_from_points(hg, orc, d, n, T, seed, prec, bias):
    """type2_batch = 1: the batched type-II sequences against the oracle's
    (batch_type2), in FP64 and with the FP32 filter."""
    w = synth.pareto_weights(n, 2.4, seed)
    x = synth.positions(n, d, seed)
    c = orc.solve_c(w, d, T, 14.0)
    ge, info, run = run_both(hg, orc, w, x, T=T, c=c, seed=seed, cl_bias=bias, type2_batch=1,
                             precision=prec)
    compare(ge, run, info=info)
    assert run.stats["seqs"] > 0
    assert info["tests"] == run.stats["tests"]
    assert info["draws"] == run.stats["draws"]
    assert info["candidates"] == run.stats["candidates"]
    assert info["type2_edges"] == run.stats["type2_edges"]


def test_batched_clustered_and_heavy(hg, orc):
    """Clustered points and heavy tails: sequences with many cell pairs, and
    from inside sequences both pairs of many candidates (queued with their own
    streams) and segmented pairs (deferred)."""
    n, d, T = 12000, 2, 0.7
    w = synth.pareto_weights(n, 2.1, 31)
    x = synth.clustered_positions(n, d, 31)
    c = orc.solve_c(w, d, T, 14.0)
    ge, info, run = run_both(hg, orc, w, x, T=T, c=c, seed=31, cl_bias=1, type2_batch=1)
    compare(ge, run, info=info)
    assert info["heavy_items"] > 0
    assert info["draws"] == run.stats["draws"]


@pytest.mark.parametrize("d,n,beta,T,seed", [(2, 2**17, 2.7, 0.5, 22), (3, 2**17, 2.3, 0.8, 23)])
def test_batched_mixed_equals_fp64(hg, d, n, beta, T, seed):
    kw = dict(d=d, beta=beta, T=T, avg_deg=16.0, seed=seed, type2_batch=1)
    a = hg.generate(n, precision=0, **kw)
    b = hg.generate(n, precision=1, **kw)
    assert np.array_equal(a.edges.cpu().numpy(), b.edges.cpu().numpy())
    assert b.info["rechecks"] > 0
    for k in ("tests", "draws", "candidates", "type1_edges", "type2_edges"):
        assert a.info[k] == b.info[k], k


def test_batched_option_where_it_does_not_apply(hg):
    """type2_batch = 1 changes nothing at d = 1, for T = 0 and for the HRG
    (no batched sequences there), and is rejected with more than 32 weight
    layers (a kept cell stores 32 bits of its layer mask)."""
    import torch
    for kw in (dict(d=1, beta=2.5, T=0.5, avg_deg=12.0, seed=41), dict(d=2, beta=2.5, T=0.0, avg_deg=12.0, seed=42)):
        a = hg.generate(30000, type2_batch=0, **kw)
        b = hg.generate(30000, type2_batch=1, **kw)
        assert torch.equal(a.edges, b.edges), kw
        assert a.info["draws"] == b.info["draws"]
    R = hg.hrg_solve_R(20000, 0.75, 0.5, 10.0)
    r = torch.from_numpy(synth.hrg_radii(20000, 0.75, R, 44)).cuda()
    xh = torch.from_numpy(np.ascontiguousarray(synth.positions(20000, 1, 44).T)).cuda()
    a = hg.from_points(r, xh, T=0.5, seed=44, model=1, R=R, alpha=0.75, type2_batch=0)
    b = hg.from_points(r, xh, T=0.5, seed=44, model=1, R=R, alpha=0.75, type2_batch=1)
    assert torch.equal(a.edges, b.edges)
    n = 4000
    w = synth.pareto_weights(n, 2.5, 43)
    w[0] = 2.0**40  # layers 0 .. 40
    x = synth.positions(n, 2, 43)
    wd = torch.from_numpy(w).cuda()
    xd = torch.from_numpy(np.ascontiguousarray(x.T)).cuda()
    with pytest.raises(hg.GirgError, match="32 weight layers"):
        hg.from_points(wd, xd, T=0.5, c=0.5, seed=43, type2_batch=1)
    ok = hg.from_points(wd, xd, T=0.5, c=0.5, seed=43, type2_batch=0)
    assert ok.edges.shape[0] > 0
