"""Calls on a caller's own stream, and concurrent calls from several host
threads (they share the library's context, whose lock serialises them):
every edge array equals the one of a plain sequential call."""
import threading

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


CASES = [dict(n=30000, d=2, beta=2.7, T=0.5, avg_deg=16.0, seed=51),
         dict(n=20000, d=1, beta=2.5, T=0.0, avg_deg=10.0, seed=52),
         dict(n=15000, d=3, beta=2.3, T=0.8, avg_deg=20.0, seed=53, precision=1),
         dict(n=25000, d=2, beta=2.2, T=0.3, avg_deg=12.0, seed=54)]


def test_user_stream(hg):
    import torch
    for case in CASES[:2]:
        ref = hg.generate(**case).edges.cpu().numpy()
        s = torch.cuda.Stream()
        with torch.cuda.stream(s):
            r = hg.generate(**case, stream=s)
        s.synchronize()
        assert np.array_equal(r.edges.cpu().numpy(), ref)
        h = hg.hrg(12000, 0.75, T=0.5, avg_deg=10.0, seed=55, stream=s)
        s.synchronize()
        assert np.array_equal(h.edges.cpu().numpy(), hg.hrg(12000, 0.75, T=0.5, avg_deg=10.0, seed=55).edges.cpu().numpy())


def test_concurrent_host_threads(hg):
    import torch
    ref = [hg.generate(**c).edges.cpu().numpy() for c in CASES]
    out = [[None] * 3 for _ in CASES]
    errs = []

    def work(k):
        try:
            s = torch.cuda.Stream()
            for rep in range(3):
                r = hg.generate(**CASES[k], stream=s)
                s.synchronize()
                out[k][rep] = r.edges.cpu().numpy()
        except Exception as e:  # reported below
            errs.append(repr(e))

    ts = [threading.Thread(target=work, args=(k,)) for k in range(len(CASES))]
    for t in ts:
        t.start()
    for t in ts:
        t.join(timeout=300)
    assert not errs, errs
    for k in range(len(CASES)):
        for rep in range(3):
            assert np.array_equal(out[k][rep], ref[k]), (k, rep)
