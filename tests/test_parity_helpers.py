"""The parity comparison itself (CPU): order-insensitive but orientation- and
content-sensitive, with the canonical key unique per edge."""
import numpy as np
import pytest

from tests import synth
from tests.parity import canonical_order, compare


@pytest.fixture(scope="module")
def run(orc):
    n, d, T = 3000, 2, 0.5
    w = synth.pareto_weights(n, 2.6, 4)
    x = synth.positions(n, d, 4)
    c = orc.solve_c(w, d, T, 14.0)
    return orc.run(w, x, T=T, c=c, seed=4, cl_bias=1, keep=True)


def test_canonical_keys_are_unique(run):
    e, keys = canonical_order(run.edges, run)
    assert len(np.unique(keys[:, :6], axis=0)) == len(keys)
    assert (keys[:, 6] == 1).any() and (keys[:, 6] == 0).any()  # both item types occur
    assert not keys[:, 7].any()


def test_compare_accepts_any_order(run):
    rng = np.random.default_rng(1)
    perm = rng.permutation(len(run.edges))
    rep = compare(run.edges[perm], run)
    assert rep["oriented"] == len(run.edges) and rep["unexplained"] == 0


def test_compare_rejects_a_flipped_edge(run):
    bad = run.edges.copy()
    bad[17] = bad[17][::-1]
    with pytest.raises(AssertionError, match="A side"):
        compare(bad, run)


def test_compare_rejects_a_missing_edge(run):
    with pytest.raises(AssertionError, match="differ"):
        compare(run.edges[1:], run)
