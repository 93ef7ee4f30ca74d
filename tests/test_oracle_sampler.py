"""Pins of the oracle's sampler against what the paper and the mathematics
fix: the plain definition of the threshold graphs (brute force over all
pairs), the coverage invariant of the cell-pair iteration, the cell-pair
counts of Fig. 7b, and the edge distribution of the binomial variants
(chi-square on per-pair frequencies, conditional mean, the T -> 0 limit)."""
import itertools
import os
from decimal import Decimal, getcontext

import numpy as np
import pytest
from scipy import stats

from tests import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def torus_linf(x):
    """All-pairs L-infinity torus distance, exact for multiples of 2^-53."""
    n, d = x.shape
    r = np.zeros((n, n))
    for k in range(d):
        dk = np.abs(x[:, None, k] - x[None, :, k])
        r = np.maximum(r, np.minimum(dk, 1.0 - dk))
    return r


def pairset(edges):
    return {(min(int(u), int(v)), max(int(u), int(v))) for u, v in edges}


def girg_p_numpy(w, x, c, T):
    """Eq. (1) evaluated for every pair, straight from the definition."""
    n, d = x.shape
    W = w.sum()
    r = torus_linf(x)
    with np.errstate(divide="ignore", over="ignore"):
        p = np.minimum(1.0, c * ((w[:, None] * w[None, :] / W) / r**d) ** (1.0 / T))
    p[r == 0] = 1.0
    np.fill_diagonal(p, 0.0)
    return p


# ---------------------------------------------------------------- threshold
@pytest.mark.parametrize("d,n,beta,seed,clustered", [
    (1, 3000, 2.5, 1, False), (2, 3000, 2.7, 2, False), (3, 2000, 2.3, 4, False),
    (2, 2000, 2.1, 9, True), (1, 2500, 3.0, 5, True),
])
def test_threshold_girg_equals_bruteforce(orc, d, n, beta, seed, clustered):
    w = synth.pareto_weights(n, beta, seed)
    x = synth.clustered_positions(n, d, seed) if clustered else synth.positions(n, d, seed)
    c = orc.solve_c(w, d, 0.0, 10.0)
    run = orc.run(w, x, T=0.0, c=c, seed=seed)
    W = w.sum()
    r = torus_linf(x)
    t = c * (w[:, None] * w[None, :] / W) ** (1.0 / d)
    iu = np.triu_indices(n, 1)
    edge = (r <= t)[iu]
    near = (np.abs(r - t) <= 1e-12 * t)[iu]
    bf = {(int(a), int(b)) for a, b, e in zip(iu[0], iu[1], edge) if e}
    amb = {(int(a), int(b)) for a, b, e in zip(iu[0], iu[1], near) if e}
    got = pairset(run.edges)
    assert len(got) == len(run.edges)  # no duplicates
    assert (got ^ bf) <= amb
    assert run.stats["type2_items"] == 0


@pytest.mark.parametrize("max_depth,cl_bias", [(0, 0), (2, 0), (-1, -1), (-1, -3)])
def test_threshold_exact_under_shallower_levels(orc, max_depth, cl_bias):
    n, d = 1500, 2
    w = synth.pareto_weights(n, 2.5, 3)
    x = synth.positions(n, d, 3)
    c = orc.solve_c(w, d, 0.0, 12.0)
    base = pairset(orc.run(w, x, T=0.0, c=c, seed=1).edges)
    alt = pairset(orc.run(w, x, T=0.0, c=c, seed=1, max_depth=max_depth, cl_bias=cl_bias).edges)
    assert base == alt


def _dec_cos(x, terms=60):
    s, t = Decimal(1), Decimal(1)
    for k in range(1, terms):
        t = -t * x * x / ((2 * k - 1) * (2 * k))
        s += t
    return s


def _dec_pi():
    # Machin: pi = 16 atan(1/5) - 4 atan(1/239)
    def atan_inv(m):
        x = Decimal(1) / m
        s, t, k = Decimal(0), x, 0
        while t != 0:
            s += t / (2 * k + 1) if k % 2 == 0 else -t / (2 * k + 1)
            t = t / (m * m)
            k += 1
        return s
    return 16 * atan_inv(Decimal(5)) - 4 * atan_inv(Decimal(239))


def test_threshold_hrg_equals_literal_formula(orc):
    """T = 0 HRG: edge iff d < R with the paper's product formula for cosh d,
    evaluated in 60-digit decimal arithmetic (free of the cancellation)."""
    getcontext().prec = 60
    n, alpha = 120, 0.75
    R = orc.hrg_solve_R(n, alpha, 0.0, 8.0)
    r = synth.hrg_radii(n, alpha, R, 7)
    x = synth.positions(n, 1, 7)
    run = orc.run(r, x, T=0.0, model=1, R=R, seed=7)
    pi = _dec_pi()
    coshR = (Decimal(R).exp() + (-Decimal(R)).exp()) / 2
    ch = [(Decimal(v).exp() + (-Decimal(v)).exp()) / 2 for v in r]
    sh = [(Decimal(v).exp() - (-Decimal(v)).exp()) / 2 for v in r]
    bf, amb = set(), set()
    for u, v in itertools.combinations(range(n), 2):
        dx = abs(Decimal(x[u, 0]) - Decimal(x[v, 0]))
        dth = 2 * pi * dx  # cos is even and 2 pi periodic: no reduction needed
        cd = ch[u] * ch[v] - sh[u] * sh[v] * _dec_cos(dth)
        if cd < coshR:
            bf.add((u, v))
        if abs(cd - coshR) <= Decimal("1e-12") * coshR:
            amb.add((u, v))
    got = pairset(run.edges)
    assert len(bf) > 50
    assert (got ^ bf) <= amb


# ---------------------------------------------------------------- coverage
@pytest.mark.parametrize("d", [1, 2, 3])
@pytest.mark.parametrize("cl_bias,max_depth", [(0, -1), (2, -1), (3, -1), (1, 1), (0, 0), (4, 2)])
def test_coverage_every_pair_exactly_once(orc, d, cl_bias, max_depth):
    """With every pair accepted, the cell-pair iteration (Algorithm 1 plus
    the double counting rules of App. B.1) visits each unordered vertex pair
    exactly once."""
    for seed, n in ((1, 40), (2, 73)):
        w = synth.pareto_weights(n, 2.2, seed)
        x = synth.clustered_positions(n, d, seed, clusters=3) if seed == 2 else synth.positions(n, d, seed)
        run = orc.run(w, x, T=0.5, c=0.3, seed=seed, cl_bias=cl_bias, max_depth=max_depth,
                      accept_all=True)
        e = run.edges
        assert len(e) == n * (n - 1) // 2
        assert len(pairset(e)) == len(e)
        assert np.all(e[:, 0] != e[:, 1])


def test_coverage_hrg(orc):
    n, alpha, R = 60, 0.8, 9.0
    r = synth.hrg_radii(n, alpha, R, 3)
    x = synth.positions(n, 1, 3)
    for bias in (0, 2):
        run = orc.run(r, x, T=0.5, model=1, R=R, seed=3, cl_bias=bias, accept_all=True)
        assert len(run.edges) == n * (n - 1) // 2 == len(pairset(run.edges))


# ---------------------------------------------------------------- Fig. 7b
def _bruteforce_cell_pairs(d, level):
    """Unordered cell pairs at a level: neighbours (every torus coordinate
    difference <= 1) and distant pairs whose parents are neighbours."""
    side = 2**level

    def tdist(a, b, s):
        df = abs(a - b)
        return min(df, s - df)

    cells = list(itertools.product(range(side), repeat=d))
    nb = dist = 0
    for a, b in itertools.combinations_with_replacement(cells, 2):
        if all(tdist(p, q, side) <= 1 for p, q in zip(a, b)):
            nb += 1
        elif all(tdist(p // 2, q // 2, side // 2) <= 1 for p, q in zip(a, b)):
            dist += 1
    return nb, dist


def test_fig7b_cell_pair_counts(orc):
    with open(os.path.join(GOLDEN, "fig7b_cell_pairs.txt")) as f:
        rows = [ln.split() for ln in f if ln.strip() and not ln.startswith("#")]
    n = 4096
    w = np.ones(n)
    x = synth.positions(n, 1, 1)
    run = orc.run(w, x, T=0.5, c=1e-6, seed=1, cl_bias=0, max_depth=5)
    assert run.stats["D"] >= 5
    for d, level, nb, dist in rows:
        level = int(level)
        assert run.level_nb[level] == int(nb)
        if dist != "NA":
            assert run.level_dist[level] == int(dist)


@pytest.mark.parametrize("d,levels", [(1, [2, 3, 4, 5]), (2, [2, 3]), (3, [2])])
def test_cell_pair_counts_bruteforce(orc, d, levels):
    n = 8192
    w = np.ones(n)
    x = synth.positions(n, d, 2)
    run = orc.run(w, x, T=0.5, c=1e-9, seed=1, max_depth=max(levels))
    for level in levels:
        nb, dist = _bruteforce_cell_pairs(d, level)
        assert run.level_nb[level] == nb
        assert run.level_dist[level] == dist
        if level >= 3 or (d == 1 and level >= 3):
            assert nb == 2 ** (level * d) * (3**d + 1) // 2
            assert dist == 2 ** (level * d) * (6**d - 3**d) // 2


# ---------------------------------------------------------------- binomial
def _freqs(orc, w, x, c, T, S, **kw):
    n = len(w)
    cnt = np.zeros((n, n))
    stats_acc = {"type2_items": 0, "candidates": 0}
    for s in range(S):
        run = orc.run(w, x, T=T, c=c, seed=1000 + s, **kw)
        e = run.edges
        cnt[e[:, 0], e[:, 1]] += 1
        for k in stats_acc:
            stats_acc[k] += run.stats[k]
    cnt = cnt + cnt.T
    return cnt, stats_acc


def _chi2_pvalue(cnt, p, S):
    iu = np.triu_indices(len(p), 1)
    obs, pp = cnt[iu], p[iu]
    mask = (pp > 0) & (pp < 1)
    # pairs with p = 1 must always be present, p = 0 never
    assert np.all(obs[pp >= 1] == S)
    assert np.all(obs[pp <= 0] == 0)
    chi = np.sum((obs[mask] - S * pp[mask]) ** 2 / (S * pp[mask] * (1 - pp[mask])))
    return stats.chi2.sf(chi, mask.sum())


@pytest.mark.parametrize("d,n,T,bias", [(1, 12, 0.5, 3), (2, 14, 0.3, 2), (3, 12, 0.8, 1), (1, 10, 0.9, 0)])
def test_binomial_girg_chi_square(orc, d, n, T, bias):
    w = synth.pareto_weights(n, 2.5, 21 + d)
    x = synth.positions(n, d, 21 + d)
    p = girg_p_numpy(w, x, 0.1, T)
    c = 0.35 / np.median(p[np.triu_indices(n, 1)]) * 0.1
    p = girg_p_numpy(w, x, c, T)
    S = 6000
    cnt, st = _freqs(orc, w, x, c, T, S, cl_bias=bias)
    assert st["type2_items"] > 0 and st["candidates"] > 0
    assert _chi2_pvalue(cnt, p, S) > 1e-4


def test_binomial_plain_bernoulli_at_depth_zero(orc):
    """max_depth = 0 puts every pair in one type-I test (a plain coin per
    pair); its frequencies obey the same law."""
    n, d, T = 12, 2, 0.5
    w = synth.pareto_weights(n, 2.5, 3)
    x = synth.positions(n, d, 3)
    c = 0.05
    p = girg_p_numpy(w, x, c, T)
    S = 4000
    cnt, st = _freqs(orc, w, x, c, T, S, max_depth=0)
    assert st["type2_items"] == 0
    assert _chi2_pvalue(cnt, p, S) > 1e-4


def test_binomial_conditional_mean(orc):
    n, d, T = 1500, 2, 0.5
    w = synth.pareto_weights(n, 2.7, 8)
    x = synth.positions(n, d, 8)
    c = orc.solve_c(w, d, T, 16.0)
    p = girg_p_numpy(w, x, c, T)
    iu = np.triu_indices(n, 1)
    mu, var = p[iu].sum(), (p[iu] * (1 - p[iu])).sum()
    S = 40
    ms = [len(orc.run(w, x, T=T, c=c, seed=s).edges) for s in range(S)]
    assert abs(np.mean(ms) - mu) < 4.5 * np.sqrt(var / S)


def test_binomial_hrg_chi_square(orc):
    n, alpha, R, T = 12, 0.75, 6.0, 0.5
    r = synth.hrg_radii(n, alpha, R, 5)
    x = synth.positions(n, 1, 5)
    dx = np.abs(x[:, None, 0] - x[None, :, 0])
    dx = np.minimum(dx, 1 - dx)
    # the paper's product formula, accurate at these small radii
    cd = np.cosh(r[:, None]) * np.cosh(r[None, :]) - np.sinh(r[:, None]) * np.sinh(r[None, :]) * np.cos(2 * np.pi * dx)
    dist = np.arccosh(np.maximum(cd, 1.0))
    p = 1.0 / (np.exp((dist - R) / (2 * T)) + 1.0)
    np.fill_diagonal(p, 0.0)
    S = 6000
    cnt = np.zeros((n, n))
    t2 = 0
    for s in range(S):
        run = orc.run(r, x, T=T, model=1, R=R, seed=500 + s, cl_bias=3)
        cnt[run.edges[:, 0], run.edges[:, 1]] += 1
        t2 += run.stats["type2_items"]
    cnt = cnt + cnt.T
    assert t2 > 0
    assert _chi2_pvalue(cnt, p, S) > 1e-4


def test_low_temperature_limit(orc):
    """T -> 0: the binomial graph with c_T = c^{d/T} approaches the threshold
    graph with c (Sec. 2.1, Sec. 1)."""
    n, d = 3000, 1
    w = synth.pareto_weights(n, 2.5, 4)
    x = synth.positions(n, d, 4)
    c = orc.solve_c(w, d, 0.0, 10.0)
    thr = pairset(orc.run(w, x, T=0.0, c=c, seed=4).edges)
    T = 0.01
    bino = pairset(orc.run(w, x, T=T, c=c ** (d / T), seed=4).edges)
    jac = len(thr & bino) / len(thr | bino)
    assert jac > 0.97


def test_power_law_degrees(orc):
    n, d, beta = 2**16, 1, 2.5
    w, x = orc.points_girg(n, d, beta, 1)
    c = orc.solve_c(w, d, 0.0, 10.0)
    run = orc.run(w, x, T=0.0, c=c, seed=1)
    deg = np.bincount(run.edges.ravel().astype(np.int64), minlength=n)
    top = np.sort(deg)[::-1][:600].astype(float)
    hill = 1.0 / np.mean(np.log(top[:-1] / top[-1]))  # CCDF exponent beta - 1
    assert abs(hill + 1.0 - beta) < 0.35


@pytest.mark.parametrize("T,d", [(0.0, 2), (0.5, 3), (0.9, 1)])
def test_coincident_points_give_the_complete_graph(orc, T, d):
    """All vertices at one position with one weight: distance 0, so p_uv = 1
    (Eq. (1) saturates) and the threshold holds for every pair: the sampler
    must return each of the n (n - 1) / 2 pairs exactly once, from a single
    type-I item (one layer, one cell at every level)."""
    n = 600
    w = np.full(n, 3.0)
    x = np.full((n, d), 0.3125)
    run = orc.run(w, x, T=T, c=0.5, seed=7, keep=True)
    e = np.sort(run.edges.astype(np.int64), axis=1)
    assert len(e) == n * (n - 1) // 2
    assert len(np.unique(e[:, 0] * n + e[:, 1])) == n * (n - 1) // 2
    assert run.stats["type1_items"] == 1 and run.stats["type2_items"] == 0


@pytest.mark.parametrize("bias", [-2, 1])
def test_binomial_edge_count_variance(orc, bias):
    """Edges are independent given the points (Sec. 2.1): over seeds, the
    number of edges has variance sum p_uv (1 - p_uv).  Coins shared between
    pairs (a Philox word used twice, a jump sequence reused) correlate pairs
    and inflate it; the mean stays sum p_uv.  cl_bias = -2 leaves nearly
    every pair to type-I tests, cl_bias = 1 most of them to type-II items."""
    n, d, T = 300, 2, 0.6
    w = synth.pareto_weights(n, 2.4, 19)
    x = synth.positions(n, d, 19)
    c = orc.solve_c(w, d, T, 12.0)
    p = girg_p_numpy(w, x, c, T)
    iu = np.triu_indices(n, 1)
    mu, var = p[iu].sum(), (p[iu] * (1 - p[iu])).sum()
    S = 1500
    ms = np.array([len(orc.run(w, x, T=T, c=c, seed=20000 + s, cl_bias=bias).edges) for s in range(S)],
                  dtype=float)
    assert abs(ms.mean() - mu) < 4.5 * np.sqrt(var / S)
    ratio = ms.var(ddof=1) / var
    lo, hi = stats.chi2.ppf([1e-5, 1 - 1e-5], S - 1) / (S - 1)
    assert lo < ratio < hi, ratio
