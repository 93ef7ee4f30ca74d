"""Pins of the oracle's type-II path on items whose candidate range is cut
into several segments, each with its own geometric-jump sequence (Sec. 3.2;
the cut is exact because the candidates are independent Bernoulli trials).

The points are fixed: groups of vertices of one weight layer in cells that are
distant at the comparison level, with an upper bound pbar large enough that an
item's range spans several segments of about 2^5 / pbar candidates.  Over many
seeds the edges between two groups must then follow Eq. (1) pair by pair
(chi-square against p_uv from the definition), be independent (the variance of
their number equals sum p_uv (1 - p_uv); segments that shared a jump sequence,
or overlapped, would correlate pairs and inflate it), and keep their mean
(sum p_uv).  A segment start or end off by one, or a jump sequence reused
across segments, fails one of these."""
import numpy as np
import pytest
from scipy import stats

from tests.test_oracle_sampler import _chi2_pvalue, girg_p_numpy


def grid_points(groups, d, seed):
    """Vertices in boxes: groups = [(count, lower corner, side)], positions
    uniform in each box as multiples of 2^-53."""
    rng = np.random.default_rng(seed)
    xs, gid = [], []
    for g, (cnt, lo, side) in enumerate(groups):
        q = rng.integers(0, int(side * 2**53), size=(cnt, d), dtype=np.int64)
        base = np.floor(np.asarray(lo, dtype=float) * 2.0**53).astype(np.int64)
        xs.append(((base + q) % 2**53).astype(np.float64) * 2.0**-53)
        gid.append(np.full(cnt, g))
    return np.concatenate(xs), np.concatenate(gid)


def one_layer_weights(n, seed):
    """Weights in [1, 1.9]: one layer (max / min below 2)."""
    return 1.0 + 0.9 * np.random.default_rng(seed + 1).random(n)


def c_for_pbar(w, d, T, gap_dist, target):
    """c at which pbar = c ((w_max^2 / W) / dist^d)^(1/T) (Eq. (1) at the
    smallest distance of two cells and the largest weights) equals target."""
    W = w.sum()
    return target / ((w.max() ** 2 / W) / gap_dist**d) ** (1.0 / T)


def bias_to_level(orc, w, x, T, c, level):
    run = orc.run(w, x, T=T, c=c, seed=0, keep=True)
    return level - int(run.CL[0, 0])


def sample(orc, w, x, T, c, bias, S, groups):
    n = len(w)
    cnt = np.zeros((n, n))
    per_seed = np.zeros((S, len(groups)))
    for s in range(S):
        e = orc.run(w, x, T=T, c=c, seed=5000 + s, cl_bias=bias).edges.astype(np.int64)
        cnt[e[:, 0], e[:, 1]] += 1
        for k, (ga, gb) in enumerate(groups):
            per_seed[s, k] = np.sum(np.isin(e[:, 0], ga) & np.isin(e[:, 1], gb)
                                    | np.isin(e[:, 0], gb) & np.isin(e[:, 1], ga))
    return cnt + cnt.T, per_seed


@pytest.mark.parametrize("d,T", [(1, 0.5), (2, 0.7)])
def test_segmented_items_chi_square_and_independence(orc, d, T):
    side = 0.125
    # level 3: A in cell 0, B two cells away (gap 1), C three away (gap 2 in d = 1)
    if d == 1:
        boxes = [(22, [0.0], side), (20, [0.25], side), (14, [0.375], side)]
    else:
        boxes = [(22, [0.0, 0.0], side), (20, [0.25, 0.125], side), (14, [0.375, 0.0], side)]
    x, gid = grid_points(boxes, d, seed=11 + d)
    n = len(x)
    w = one_layer_weights(n, 11 + d)
    c = c_for_pbar(w, d, T, side, 0.25)
    bias = bias_to_level(orc, w, x, T, c, 3)
    run = orc.run(w, x, T=T, c=c, seed=1, cl_bias=bias, keep=True)
    assert run.CL[0, 0] == 3
    # items of A x B span 22 * 20 = 440 candidates; pbar ~ 0.25 gives 2^7 per segment
    assert run.stats["segments"] >= run.stats["type2_items"] + 3
    p = girg_p_numpy(w, x, c, T)
    A, B, C = (np.flatnonzero(gid == k) for k in range(3))
    S = 6000
    cnt, per = sample(orc, w, x, T, c, bias, S, [(A, B), (A, C)])
    assert _chi2_pvalue(cnt, p, S) > 1e-4
    for k, (ga, gb) in enumerate([(A, B), (A, C)]):
        pp = p[np.ix_(ga, gb)]
        mu, var = pp.sum(), (pp * (1 - pp)).sum()
        m = per[:, k]
        assert abs(m.mean() - mu) < 4.5 * np.sqrt(var / S)
        # independent edges: sample variance / sum p (1 - p) ~ chi2(S-1) / (S-1)
        ratio = m.var(ddof=1) / var
        lo, hi = stats.chi2.ppf([1e-5, 1 - 1e-5], S - 1) / (S - 1)
        assert lo < ratio < hi, (k, ratio)


def test_many_segments_mean_and_variance(orc):
    """Two dense groups of 500 and 400 vertices in distant cells: one item of
    2 * 10^5 candidates cut into thousands of segments (the cap of 2^12
    segments per item raises the segment size).  Mean and variance of the
    number of edges between the groups over seeds."""
    d, T, side = 1, 0.6, 0.125
    x, gid = grid_points([(500, [0.0], side), (400, [0.25], side)], d, seed=3)
    w = one_layer_weights(len(x), 3)
    c = c_for_pbar(w, d, T, side, 0.6)
    bias = bias_to_level(orc, w, x, T, c, 3)
    run = orc.run(w, x, T=T, c=c, seed=1, cl_bias=bias, keep=True)
    assert run.stats["segments"] > run.stats["type2_items"] + 1000
    p = girg_p_numpy(w, x, c, T)
    A, B = np.flatnonzero(gid == 0), np.flatnonzero(gid == 1)
    pp = p[np.ix_(A, B)]
    mu, var = pp.sum(), (pp * (1 - pp)).sum()
    S = 400
    sizes = np.zeros(S)
    inA = np.zeros(len(x), dtype=bool)
    inA[A] = True
    for s in range(S):
        e = orc.run(w, x, T=T, c=c, seed=9000 + s, cl_bias=bias).edges.astype(np.int64)
        sizes[s] = np.sum(inA[e[:, 0]] != inA[e[:, 1]])
    assert abs(sizes.mean() - mu) < 4.5 * np.sqrt(var / S)
    ratio = sizes.var(ddof=1) / var
    lo, hi = stats.chi2.ppf([1e-5, 1 - 1e-5], S - 1) / (S - 1)
    assert lo < ratio < hi, ratio
