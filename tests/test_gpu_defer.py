"""The deferred-item lists (split type-I items, segmented type-II items) start
at a first capacity and, when one overflows, the sampling passes run once more
with exact sizes.  A tiny first capacity (GIRG_DEFER_CAPACITY) forces that
rerun: the edge array and every counter equal those of a call that needed no
rerun."""
import os

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def hg():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1905_06706_amd as hg
    hg.load()
    return hg


@pytest.mark.parametrize("case", [dict(n=40000, d=2, beta=2.4, T=0.5, avg_deg=24.0, seed=61),
                                  dict(n=30000, d=3, beta=2.2, T=0.8, avg_deg=20.0, seed=62, precision=1),
                                  dict(n=50000, d=1, beta=2.3, T=0.0, avg_deg=30.0, seed=63)])
def test_deferred_lists_grown(hg, case):
    ref = hg.generate(**case)
    assert ref.info["split_items"] + ref.info["heavy_items"] > 16
    os.environ["GIRG_DEFER_CAPACITY"] = "16"
    try:
        r = hg.generate(**case)
    finally:
        del os.environ["GIRG_DEFER_CAPACITY"]
    assert np.array_equal(r.edges.cpu().numpy(), ref.edges.cpu().numpy())
    for k in ("m", "tests", "draws", "candidates", "rechecks", "split_items", "heavy_items"):
        assert r.info[k] == ref.info[k], k
