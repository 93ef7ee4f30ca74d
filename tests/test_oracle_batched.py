"""Pins of the oracle's batched type-II sampling (one geometric-jump sequence
over the distant cell pairs of a source cell that share the bound pbar): the
same pins as the per-cell-pair sampling (Sec. 3.2, Eq. (1)), on graphs whose
comparison levels are pushed down so that many sequences of several cell
pairs occur at levels >= 3."""
import numpy as np
import pytest
from scipy import stats

from tests import synth
from tests.test_oracle_sampler import _chi2_pvalue, girg_p_numpy, pairset


@pytest.mark.parametrize("d", [2, 3])
def test_batched_coverage_every_pair_exactly_once(orc, d):
    """pbar = 1 and every candidate accepted: every unordered vertex pair is
    emitted once, and the sequences hold several cell pairs."""
    for seed, n, bias in ((1, 60, 4), (2, 90, 6)):
        w = synth.pareto_weights(n, 2.2, seed)
        x = synth.positions(n, d, seed)
        run = orc.run(w, x, T=0.5, c=0.3, seed=seed, cl_bias=bias, accept_all=True, batch_type2=True)
        e = run.edges
        assert len(e) == n * (n - 1) // 2 == len(pairset(e))
        assert np.all(e[:, 0] != e[:, 1])
        assert run.stats["seqs"] > 0
        assert run.stats["type2_items"] > 1.5 * run.stats["seqs"]


def _batched_freqs(orc, w, x, c, T, S, **kw):
    n = len(w)
    cnt = np.zeros((n, n))
    acc = {"seqs": 0, "type2_items": 0, "candidates": 0}
    for s in range(S):
        run = orc.run(w, x, T=T, c=c, seed=3000 + s, batch_type2=True, **kw)
        e = run.edges
        cnt[e[:, 0], e[:, 1]] += 1
        for k in acc:
            acc[k] += run.stats[k]
    return cnt + cnt.T, acc


@pytest.mark.parametrize("d,n,T,bias", [(2, 16, 0.4, 4), (2, 24, 0.7, 3), (3, 40, 0.8, 3)])
def test_batched_chi_square(orc, d, n, T, bias):
    """Per-pair edge frequencies over many seeds against p_uv of Eq. (1)."""
    w = synth.pareto_weights(n, 2.5, 40 + d)
    x = synth.positions(n, d, 40 + d)
    p = girg_p_numpy(w, x, 0.1, T)
    c = 0.3 / np.median(p[np.triu_indices(n, 1)]) * 0.1
    p = girg_p_numpy(w, x, c, T)
    S = 6000
    cnt, acc = _batched_freqs(orc, w, x, c, T, S, cl_bias=bias)
    assert acc["seqs"] > 0 and acc["candidates"] > 0
    assert acc["type2_items"] > 1.5 * acc["seqs"]
    assert _chi2_pvalue(cnt, p, S) > 1e-4


def test_batched_edge_count_variance_and_mean(orc):
    """Edges stay independent given the points: over seeds the edge count has
    mean sum p_uv and variance sum p_uv (1 - p_uv).  A jump sequence shared by
    two sequences, or a candidate counted in two items, shows up here."""
    n, d, T = 300, 2, 0.6
    w = synth.pareto_weights(n, 2.4, 19)
    x = synth.positions(n, d, 19)
    c = orc.solve_c(w, d, T, 12.0)
    p = girg_p_numpy(w, x, c, T)
    iu = np.triu_indices(n, 1)
    mu, var = p[iu].sum(), (p[iu] * (1 - p[iu])).sum()
    S = 1500
    seqs = 0
    ms = []
    for s in range(S):
        run = orc.run(w, x, T=T, c=c, seed=40000 + s, cl_bias=2, batch_type2=True)
        ms.append(len(run.edges))
        seqs += run.stats["seqs"]
    ms = np.array(ms, dtype=float)
    assert seqs > 0
    assert abs(ms.mean() - mu) < 4.5 * np.sqrt(var / S)
    ratio = ms.var(ddof=1) / var
    lo, hi = stats.chi2.ppf([1e-5, 1 - 1e-5], S - 1) / (S - 1)
    assert lo < ratio < hi, ratio


def test_batched_conditional_mean_and_draws(orc):
    """At a realistic size the batched graph has the expected edge count, and
    it needs far fewer draws than one sequence per cell pair."""
    n, d, T = 4000, 3, 0.8
    w = synth.pareto_weights(n, 2.3, 8)
    x = synth.positions(n, d, 8)
    c = orc.solve_c(w, d, T, 20.0)
    p = girg_p_numpy(w, x, c, T)
    iu = np.triu_indices(n, 1)
    mu, var = p[iu].sum(), (p[iu] * (1 - p[iu])).sum()
    S = 24
    ms, draws_b, draws_p = [], 0, 0
    for s in range(S):
        rb = orc.run(w, x, T=T, c=c, seed=s, batch_type2=True)
        ms.append(len(rb.edges))
        draws_b += rb.stats["draws"]
        draws_p += orc.run(w, x, T=T, c=c, seed=s).stats["draws"]
    assert abs(np.mean(ms) - mu) < 4.5 * np.sqrt(var / S)
    assert draws_b < 0.6 * draws_p


@pytest.mark.parametrize("d,T", [(2, 0.5), (3, 0.8)])
def test_batched_split_runs_equal_plain_run(orc, d, T):
    """Runs split by the level-3 ancestor (of the A side for cell pairs, of the
    source cell for sequences) together sample the plain run's graph."""
    from tests.oracle_pool import run_whole
    n = 5000
    w = synth.pareto_weights(n, 2.3, 5)
    x = synth.positions(n, d, 5)
    c = orc.solve_c(w, d, T, 16.0)
    plain = orc.run(w, x, T=T, c=c, seed=9, batch_type2=True)
    split = run_whole(w, x, level=3, nparts=5, nproc=2, T=T, c=c, seed=9, batch_type2=True)

    def okeys(e):
        e = np.asarray(e, dtype=np.uint64).reshape(-1, 2)
        return np.sort((e[:, 0] << np.uint64(32)) | e[:, 1])

    assert plain.stats["seqs"] > 0
    assert np.array_equal(okeys(split.edges), okeys(plain.edges))
    for k in ("draws", "candidates"):
        assert split.stats[k] == plain.stats[k], k


def test_batching_applies_to_girg_d2_d3_only(orc):
    """At d = 1 (one distant cell per gap) and for the HRG the option changes
    nothing: the same edges from the same per-cell-pair streams."""
    n = 3000
    w = synth.pareto_weights(n, 2.5, 6)
    x = synth.positions(n, 1, 6)
    c = orc.solve_c(w, 1, 0.5, 10.0)
    a = orc.run(w, x, T=0.5, c=c, seed=2)
    b = orc.run(w, x, T=0.5, c=c, seed=2, batch_type2=True)
    assert b.stats["seqs"] == 0
    assert np.array_equal(a.edges, b.edges)
