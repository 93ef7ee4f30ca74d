"""girg_from_points_noalloc (the entry point that allocates nothing: its
device buffers lie in a fixed array) against girg_from_points, through the C
ABI, on two calls in a row, the second with a smaller input: equal edge
arrays and counters.  Also its limits."""
import numpy as np
import pytest

from tests import synth

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


def one_case(hg, n, d, T, seed, **kw):
    import torch
    w = synth.pareto_weights(n, 2.5, seed)
    x = synth.positions(n, d, seed)
    c = hg.solve_c(w, d, T, 14.0)
    wd, xd = dev(w), dev(x.T)
    ref = hg.from_points(wd, xd, T=T, c=c, seed=seed, **kw)
    cap = ref.edges.shape[0] + 1000
    buf = torch.full((cap, 2), -1, dtype=torch.int32, device="cuda")
    m, info = hg.from_points_noalloc(wd, xd, buf, T=T, c=c, seed=seed, **kw)
    print(f"[noalloc] n={n} d={d} T={T} m={m}", flush=True)
    assert m == ref.edges.shape[0]
    assert torch.equal(buf[:m], ref.edges)
    for k in ("tests", "draws", "candidates", "rechecks", "type1_edges", "type2_edges", "near_boundary",
              "skip_ties", "L", "D", "c"):
        assert info[k] == ref.info[k], k


def test_noalloc_equals_from_points_twice(hg):
    # the second call is smaller and reuses the array the first one left
    one_case(hg, 200000, 2, 0.5, 3)
    one_case(hg, 30000, 3, 0.8, 4, precision=1)


def test_noalloc_batched_type2(hg):
    # the batched type-II sequences use the array's own offset tables
    one_case(hg, 60000, 3, 0.8, 6, type2_batch=1)
    one_case(hg, 20000, 2, 0.5, 7, precision=1, type2_batch=1)


def test_noalloc_threshold_and_hrg(hg):
    one_case(hg, 50000, 1, 0.0, 5)
    import torch
    n, alpha, T = 20000, 0.75, 0.5
    R = hg.hrg_solve_R(n, alpha, T, 10.0)
    r = dev(synth.hrg_radii(n, alpha, R, 3))
    x = dev(synth.positions(n, 1, 3).T)
    ref = hg.from_points(r, x, T=T, seed=3, model=1, R=R, alpha=alpha)
    buf = torch.empty((ref.edges.shape[0] + 10, 2), dtype=torch.int32, device="cuda")
    m, info = hg.from_points_noalloc(r, x, buf, T=T, seed=3, model=1, R=R, alpha=alpha)
    assert m == ref.edges.shape[0] and torch.equal(buf[:m], ref.edges)


def test_noalloc_limits(hg):
    import torch
    w = dev(np.ones(16))
    x = dev(synth.positions(16, 2, 1).T)
    buf = torch.empty((16, 2), dtype=torch.int32, device="cuda")
    with pytest.raises(hg.GirgError, match="c > 0"):
        hg.from_points_noalloc(w, x, buf, T=0.5, c=0.0, seed=1)
    big = dev(np.ones((1 << 20) + 1))
    bx = torch.zeros((2, (1 << 20) + 1), dtype=torch.float64, device="cuda")
    with pytest.raises(hg.GirgError, match="2\\^20"):
        hg.from_points_noalloc(big, bx, buf, T=0.5, c=0.1, seed=1)
    # overflow reports the count needed, as girg_from_points does
    w = dev(synth.pareto_weights(3000, 2.5, 2))
    x = dev(synth.positions(3000, 2, 2).T)
    with pytest.raises(hg.GirgError, match="EOVERFLOW"):
        hg.from_points_noalloc(w, x, buf, T=0.5, c=0.5, seed=2)
