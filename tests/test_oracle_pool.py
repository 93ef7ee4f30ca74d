"""The split oracle run (tests/oracle_pool.py) samples the same graph as one
plain run: the union of the top-level run and the subtree runs holds the same
oriented edges, near-boundary pairs and tie items, and the same counts of
tests, draws and candidates."""
import numpy as np
import pytest

import oracle
from tests import synth
from tests.oracle_pool import run_whole


@pytest.mark.parametrize("d,T,level,nparts", [(2, 0.5, 3, 5), (3, 0.8, 2, 4), (1, 0.0, 3, 3)])
def test_split_run_equals_plain_run(d, T, level, nparts):
    n = 6000
    w = synth.pareto_weights(n, 2.3, 3)
    x = synth.positions(n, d, 3)
    c = oracle.solve_c(w, d, T, 14.0)
    plain = oracle.run(w, x, T=T, c=c, seed=5)
    split = run_whole(w, x, level=level, nparts=nparts, nproc=2, T=T, c=c, seed=5)

    def okeys(e):
        e = np.asarray(e, dtype=np.uint64).reshape(-1, 2)
        return np.sort((e[:, 0] << np.uint64(32)) | e[:, 1])

    assert len(split.edges) == len(plain.edges)
    assert np.array_equal(okeys(split.edges), okeys(plain.edges))
    assert np.array_equal(okeys(split.near), okeys(plain.near))
    assert sorted(map(tuple, split.ties.tolist())) == sorted(map(tuple, plain.ties.tolist()))
    for k in ("tests", "draws", "candidates"):
        assert split.stats[k] == plain.stats[k], k
    assert np.array_equal(split.sorted_ids, plain.sorted_ids)
