"""Pins of the oracle's primitives: Philox4x32-10, the 53-bit uniforms, the
Morton code and the point generators."""
import os

import numpy as np
import pytest
from scipy import stats

from tests import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _rows(name):
    with open(os.path.join(GOLDEN, name)) as f:
        return [ln.split() for ln in f if ln.strip() and not ln.startswith("#")]


def test_philox_known_answers(orc):
    for row in _rows("philox4x32_10_kat.txt"):
        vals = [int(v, 16) for v in row]
        out = orc.philox4x32_10(vals[0:4], vals[4:6])
        assert list(out) == vals[6:10]


def test_philox_is_a_bijection_of_the_counter(orc):
    # different counters under one key never collide on a small sample
    seen = set()
    for c0 in range(2000):
        seen.add(tuple(orc.philox4x32_10([c0, 7, 0, 0], [1, 2])))
    assert len(seen) == 2000


def test_uniform_conversions(orc):
    assert orc.u53(0, 0) == 0.0
    assert orc.u53(0xFFFFFFFF, 0xFFFFFFFF) == 1.0 - 2.0**-53
    assert orc.u53_open(0, 0) == 2.0**-53
    assert orc.u53_open(0xFFFFFFFF, 0xFFFFFFFF) == 1.0
    # the low 11 bits of the 64-bit word are dropped
    assert orc.u53(0x7FF, 0) == 0.0
    assert orc.u53(0x800, 0) == 2.0**-53


def test_morton_paper_example(orc):
    for d, bits, a, b, code in _rows("morton_example.txt"):
        coords = [int(a, 2), int(b, 2)]
        assert orc.morton_encode(coords, int(d), int(bits)) == int(code, 2)
        assert list(orc.morton_decode(int(code, 2), int(d), int(bits))) == coords


@pytest.mark.parametrize("d", [1, 2, 3, 4])
def test_morton_bruteforce_and_roundtrip(orc, d):
    bits = 32 // d
    rng = np.random.default_rng(d)
    for _ in range(200):
        coords = rng.integers(0, 2**bits, size=d)
        # brute force: bit b of coordinate k goes to position b*d + (d-1-k)
        want = 0
        for k in range(d):
            for b in range(bits):
                if (int(coords[k]) >> b) & 1:
                    want |= 1 << (b * d + (d - 1 - k))
        code = orc.morton_encode(coords, d, bits)
        assert code == want
        assert list(orc.morton_decode(code, d, bits)) == list(coords)


def test_morton_descendants_are_consecutive(orc):
    # Sec. 3.4 property (I): the descendants of a cell form a contiguous range
    d, bits = 2, 4
    codes = {}
    for a in range(16):
        for b in range(16):
            codes[(a, b)] = orc.morton_encode([a, b], d, bits)
    for level in range(bits + 1):
        sh = bits - level
        groups = {}
        for (a, b), c in codes.items():
            groups.setdefault((a >> sh, b >> sh), []).append(c)
        for cell, cs in groups.items():
            cs = sorted(cs)
            assert cs[-1] - cs[0] + 1 == len(cs)
            parent = orc.morton_encode([cell[0], cell[1]], d, level)
            assert cs[0] >> (d * sh) == parent


def test_girg_weights_are_pareto(orc):
    beta = 2.5
    w, x = orc.points_girg(50000, 2, beta, 11)
    assert w.min() >= 1.0
    # P(w > t) = t^{-(beta-1)}: KS against the exact law
    ks = stats.kstest(w, lambda t: 1.0 - t ** (-(beta - 1.0)))
    assert ks.pvalue > 1e-3
    # positions are exact multiples of 2^-53 in [0,1)
    q = x * 2.0**53
    assert np.all(q == np.floor(q)) and np.all(x >= 0) and np.all(x < 1)
    for k in range(2):
        assert stats.kstest(x[:, k], "uniform").pvalue > 1e-3


def test_girg_points_are_deterministic_per_id(orc):
    w1, x1 = orc.points_girg(100, 3, 2.3, 5)
    w2, x2 = orc.points_girg(300, 3, 2.3, 5)
    assert np.array_equal(w1, w2[:100]) and np.array_equal(x1, x2[:100])


def test_hrg_radii_law(orc):
    alpha, R = 0.75, 20.0
    r, x = orc.points_hrg(50000, alpha, R, 3)
    assert r.min() >= 0 and r.max() <= R
    cdf = lambda t: (np.cosh(alpha * np.minimum(t, R)) - 1.0) / (np.cosh(alpha * R) - 1.0)
    assert stats.kstest(r, cdf).pvalue > 1e-3
    assert stats.kstest(x[:, 0], "uniform").pvalue > 1e-3
    # power-law exponent of the mapped weights w = exp((R - r)/2) is 2 alpha + 1
    # (Sec. 2.2): P(w > t) = t^{-2 alpha} away from the boundary
    w = np.exp((R - r) / 2.0)
    for t in (4.0, 16.0):
        emp = np.mean(w > t)
        want = t ** (-2.0 * alpha)
        assert abs(emp - want) < 5 * np.sqrt(want / len(w)) + 0.002


def test_synth_inputs_are_exact_multiples():
    x = synth.positions(1000, 3, 1)
    q = x * 2.0**53
    assert np.all(q == np.floor(q))
    xc = synth.clustered_positions(1000, 2, 1)
    assert np.all(xc >= 0) and np.all(xc < 1)
