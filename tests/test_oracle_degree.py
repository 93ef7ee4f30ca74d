"""Pins of the average-degree machinery: f(c) of App. B.2 against the
expectation of the model written out pair by pair (numerical integration of
Eq. (1) over the law of the torus distance), the ball volume (2t)^d, the
solver, and the HRG radius solve against Monte Carlo."""
import numpy as np
import pytest
from scipy import integrate

from tests import synth


def pair_expectation(wu, wv, W, c, d, T):
    """E[X_uv] for independent uniform positions: integrate the edge
    probability against the density d 2^d r^{d-1} of the torus distance on
    [0, 1/2] (P(||x_u - x_v|| <= t) = (2t)^d)."""
    X = wu * wv / W
    if T == 0.0:
        t = c * X ** (1.0 / d)
        return min(1.0, (2.0 * t) ** d)
    dens = lambda r: d * 2.0**d * r ** (d - 1)
    prob = lambda r: min(1.0, c * (X / r**d) ** (1.0 / T)) if r > 0 else 1.0
    # p = 1 below the radius k where it saturates
    k = (c**T * X) ** (1.0 / d)
    if k >= 0.5:
        return 1.0
    head = (2.0 * k) ** d
    tail, _ = integrate.quad(lambda r: prob(r) * dens(r), k, 0.5, epsabs=1e-14, epsrel=1e-12, limit=200)
    return head + tail


@pytest.mark.parametrize("d,T", [(1, 0.0), (2, 0.0), (3, 0.0), (1, 0.5), (2, 0.3), (3, 0.8)])
def test_expected_degree_matches_pairwise_integral(orc, d, T):
    n = 36
    w = synth.pareto_weights(n, 2.2, 17) * 3.0
    W = w.sum()
    for c in (0.05, 0.8, 4.0):
        want = 0.0
        for u in range(n):
            for v in range(n):
                if u != v:
                    want += pair_expectation(w[u], w[v], W, c, d, T)
        want /= n
        got = orc.expected_avg_degree(w, d, T, c)
        assert got == pytest.approx(want, rel=1e-8, abs=1e-12)


@pytest.mark.parametrize("d,T", [(1, 0.3), (2, 0.2), (1, 0.0)])
def test_expected_degree_heavy_tail(orc, d, T):
    """beta close to 2 and low temperature, where the closed form summed over
    all pairs exceeds the degree by orders of magnitude before the E_R
    correction: the pairwise sum must still be matched closely."""
    n = 60
    w = synth.pareto_weights(n, 2.05, 23) * 5.0
    W = w.sum()
    for c in (0.3, 2.0, 9.0):
        want = 0.0
        for u in range(n):
            for v in range(n):
                if u != v:
                    want += pair_expectation(w[u], w[v], W, c, d, T)
        want /= n
        got = orc.expected_avg_degree(w, d, T, c)
        assert got == pytest.approx(want, rel=1e-9, abs=1e-12)


def test_ball_volume_monte_carlo():
    # P(||x_u - x_v|| <= t) = (2t)^d on the torus (App. B.2)
    rng = np.random.default_rng(0)
    for d in (1, 2, 3):
        a, b = rng.random((400000, d)), rng.random((400000, d))
        df = np.abs(a - b)
        r = np.max(np.minimum(df, 1 - df), axis=1)
        for t in (0.05, 0.2, 0.45):
            emp = np.mean(r <= t)
            want = (2 * t) ** d
            assert abs(emp - want) < 5 * np.sqrt(want * (1 - want) / len(r))


@pytest.mark.parametrize("d,T,deg", [(1, 0.0, 10.0), (2, 0.5, 16.0), (3, 0.8, 20.0), (2, 0.3, 8.0)])
def test_solve_c_hits_target(orc, d, T, deg):
    w = synth.pareto_weights(20000, 2.5, 3)
    c = orc.solve_c(w, d, T, deg)
    assert orc.expected_avg_degree(w, d, T, c) == pytest.approx(deg, rel=1e-9)
    # monotone in c
    assert orc.expected_avg_degree(w, d, T, c * 1.01) > deg > orc.expected_avg_degree(w, d, T, c * 0.99)


@pytest.mark.parametrize("d,T,deg", [(1, 0.0, 10.0), (2, 0.5, 16.0), (3, 0.8, 20.0)])
def test_realised_degree_matches_target(orc, d, T, deg):
    n = 8000
    w = synth.pareto_weights(n, 2.6, 4)
    c = orc.solve_c(w, d, T, deg)
    degs = []
    for s in range(12):
        x = synth.positions(n, d, 100 + s)
        degs.append(2.0 * len(orc.run(w, x, T=T, c=c, seed=s).edges) / n)
    # the only randomness left is positions and coins; heavy vertices make the
    # spread wider than Poisson, so allow 3 standard errors plus 1 %
    se = np.std(degs) / np.sqrt(len(degs))
    assert abs(np.mean(degs) - deg) < 3 * se + 0.01 * deg


def test_hrg_expected_degree_monte_carlo(orc):
    n, alpha, T, R = 5000, 0.75, 0.5, 16.0
    rng = np.random.default_rng(2)
    M = 400000
    u1, u2 = rng.random(M), rng.random(M)
    cm = np.cosh(alpha * R) - 1
    r1 = np.arccosh(1 + u1 * cm) / alpha
    r2 = np.arccosh(1 + u2 * cm) / alpha
    phi = rng.random(M) * np.pi
    cd = np.cosh(r1 - r2) + 2 * np.sinh(r1) * np.sinh(r2) * np.sin(phi / 2) ** 2
    p = 1.0 / (np.exp((np.arccosh(cd) - R) / (2 * T)) + 1.0)
    mc = (n - 1) * p.mean()
    se = (n - 1) * p.std() / np.sqrt(M)
    got = orc.hrg_expected_avg_degree(n, alpha, T, R)
    assert abs(got - mc) < 5 * se


def test_hrg_threshold_expected_degree_monte_carlo(orc):
    n, alpha, R = 3000, 0.8, 15.0
    rng = np.random.default_rng(3)
    M = 400000
    cm = np.cosh(alpha * R) - 1
    r1 = np.arccosh(1 + rng.random(M) * cm) / alpha
    r2 = np.arccosh(1 + rng.random(M) * cm) / alpha
    phi = rng.random(M) * np.pi
    cd = np.cosh(r1 - r2) + 2 * np.sinh(r1) * np.sinh(r2) * np.sin(phi / 2) ** 2
    p = (cd < np.cosh(R)).astype(float)
    mc, se = (n - 1) * p.mean(), (n - 1) * p.std() / np.sqrt(M)
    assert abs(orc.hrg_expected_avg_degree(n, alpha, 0.0, R) - mc) < 5 * se


def test_hrg_solve_R_realised(orc):
    n, alpha, T, deg = 4000, 0.75, 0.5, 10.0
    R = orc.hrg_solve_R(n, alpha, T, deg)
    assert orc.hrg_expected_avg_degree(n, alpha, T, R) == pytest.approx(deg, rel=1e-9)
    degs = []
    for s in range(10):
        r, x = orc.points_hrg(n, alpha, R, 40 + s)
        degs.append(2.0 * len(orc.run(r, x, T=T, model=1, R=R, seed=s).edges) / n)
    se = np.std(degs) / np.sqrt(len(degs))
    assert abs(np.mean(degs) - deg) < 3 * se + 0.02 * deg
