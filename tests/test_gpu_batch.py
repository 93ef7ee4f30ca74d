"""girg_generate_batch: instances run concurrently on the library's worker
streams; every instance's edges and counters must equal those of a single
call with the same parameters, in instance order."""
import ctypes

import numpy as np
import pytest

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


def mixed_params(hg):
    P = []
    rng = np.random.default_rng(11)
    for b in range(18):
        n = int(rng.integers(300, 40000))
        d = 1 + b % 4
        T = [0.0, 0.3, 0.9][b % 3]
        prec = 1 if b % 5 == 4 else 0
        P.append(hg.make_params(n, d, float(rng.uniform(2.1, 3.0)), T, float(rng.uniform(6, 24)), 0.0,
                                500 + b, prec))
    # HRGs: R solved from the degree, and R given
    P.append(hg.make_params(20000, 1, 0.0, 0.5, 10.0, 0.0, 77, model=1, alpha=0.75))
    P.append(hg.make_params(5000, 1, 0.0, 0.0, 0.0, 0.0, 78, model=1, alpha=0.9, R=14.0))
    return P


def single(hg, p):
    if p.model == 1:
        return hg.hrg(p.n, p.alpha, T=p.T, R=p.R, avg_deg=p.avg_deg, seed=p.seed)
    return hg.generate(p.n, d=p.d, beta=p.beta, T=p.T, avg_deg=p.avg_deg, seed=p.seed,
                       precision=p.precision)


def test_batch_matches_single_calls(hg):
    P = mixed_params(hg)
    print(f"[batch] {len(P)} instances", flush=True)
    edges, offs, infos = hg.generate_batch(P)
    assert offs[0] == 0 and offs[-1] == edges.shape[0]
    e = edges.cpu().numpy()
    for b, p in enumerate(P):
        s = single(hg, p)
        assert np.array_equal(e[offs[b]:offs[b + 1]], s.edges.cpu().numpy()), b
        for k in ("m", "tests", "draws", "candidates", "rechecks", "type1_edges", "type2_edges"):
            assert infos[b][k] == s.info[k], (b, k)


def test_batch_is_repeatable(hg):
    P = mixed_params(hg)[:12]
    a, oa, _ = hg.generate_batch(P)
    b, ob, _ = hg.generate_batch(P)
    assert oa == ob
    assert np.array_equal(a.cpu().numpy(), b.cpu().numpy())


def test_batch_overflow_reports_total(hg):
    import torch
    P = mixed_params(hg)[:8]
    _, offs, _ = hg.generate_batch(P)
    L = hg.load()
    arr = (hg.Params * len(P))(*P)
    buf = torch.empty((16, 2), dtype=torch.int32, device="cuda")
    o = (ctypes.c_uint64 * (len(P) + 1))()
    st = L.girg_generate_batch(arr, len(P), ctypes.c_void_p(buf.data_ptr()), 16, o, None,
                               ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert st == hg.GIRG_EOVERFLOW
    assert o[len(P)] == offs[-1]


def test_batch_invalid_instance(hg):
    P = mixed_params(hg)[:4]
    P[2] = hg.make_params(1000, 5, 2.5, 0.0, 10.0, 0.0, 1)  # d = 5
    with pytest.raises(hg.GirgError, match="instance 2"):
        hg.generate_batch(P)


def test_batch_recipe_against_oracle(hg, orc):
    """A reduced version of the 256-instance benchmark recipe (n up to ~3e4);
    every fourth instance is checked against the oracle."""
    rng = np.random.default_rng(5)
    P = []
    for b in range(64):
        n = int(round(10 ** (3 + 1.5 * rng.random())))
        P.append(hg.make_params(n, int(rng.integers(1, 3)), float(rng.uniform(2.1, 3.0)),
                                float(rng.choice([0.0, 0.3, 0.9])), float(rng.uniform(8, 32)), 0.0,
                                1000 + b))
    edges, offs, infos = hg.generate_batch(P)
    e = edges.cpu().numpy().view(np.uint32)
    for b in range(0, len(P), 4):
        p = P[b]
        w, x = orc.points_girg(p.n, p.d, p.beta, p.seed)
        c = orc.solve_c(w, p.d, p.T, p.avg_deg)
        assert infos[b]["c"] == pytest.approx(c, rel=1e-12)
        run = orc.run(w, x, T=p.T, c=c, seed=p.seed, keep=True)
        compare(e[offs[b]:offs[b + 1]], run)


def test_batch_full_recipe_largest_against_oracle(hg, orc):
    """The benchmark's 256-instance recipe at its real sizes (n up to 10^6),
    FP32 filter with FP64 recheck (the reported leg): equal to the FP64 batch
    bit for bit, and its three largest instances plus three others against the
    oracle on the GPU's points and constants."""
    import bench
    from tests.parity import compare_large
    Pm = bench.batch_params(hg, dict(batch=256, master_seed=5), 1)
    Pf = bench.batch_params(hg, dict(batch=256, master_seed=5), 0)
    print(f"[batch] recipe: {len(Pm)} instances, n total {sum(p.n for p in Pm)}", flush=True)
    em, om, im = hg.generate_batch(Pm)
    ef, of, _ = hg.generate_batch(Pf)
    assert om == of
    import torch
    assert torch.equal(em, ef)
    e = em.cpu().numpy().view(np.uint32)
    del ef
    order = sorted(range(len(Pm)), key=lambda b: -Pm[b].n)
    pick = order[:3] + order[60:256:80]
    for b in pick:
        p = Pm[b]
        print(f"[batch] instance {b}: n={p.n} d={p.d} beta={p.beta:.3f} T={p.T} deg={p.avg_deg:.2f}",
              flush=True)
        wd, xd = hg.points(p.n, p.d, p.beta, seed=p.seed)
        w, x = wd.cpu().numpy(), np.ascontiguousarray(xd.cpu().numpy().T)
        assert im[b]["c"] == pytest.approx(orc.solve_c(w, p.d, p.T, p.avg_deg), rel=1e-12)
        run = orc.run(w, x, T=p.T, c=im[b]["c"], seed=p.seed, keep=True)
        rep = compare_large(e[om[b]:om[b + 1]], run, info=im[b])
        assert rep["gpu"] == om[b + 1] - om[b]
        run.close()


def test_batch_waits_for_the_callers_stream(hg):
    """Work queued on the caller's stream before the call (here a long chain of
    kernels that ends by filling the edge buffer with -1) finishes before any
    instance writes an edge: the batch's workers wait for that stream."""
    import torch
    P = mixed_params(hg)[:6]
    ref, roffs, _ = hg.generate_batch(P)
    total = roffs[-1]
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        buf = torch.empty((total, 2), dtype=torch.int32, device="cuda")
        x = torch.ones(1 << 26, device="cuda")
        for _ in range(40):
            x = x * 1.0001 + 0.5
        buf.fill_(-1)
    L = hg.load()
    arr = (hg.Params * len(P))(*P)
    offs = (ctypes.c_uint64 * (len(P) + 1))()
    st = L.girg_generate_batch(arr, len(P), ctypes.c_void_p(buf.data_ptr()), total, offs, None,
                               ctypes.c_void_p(s.cuda_stream))
    assert st == hg.GIRG_OK
    torch.cuda.synchronize()
    assert list(offs) == roffs
    assert torch.equal(buf, ref)
    del x
