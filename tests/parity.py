"""Comparison helpers for GPU-vs-oracle parity: edge sets must be equal except
for pairs the oracle logged as near the decision boundary (|U - p| < 1e-12,
or a relative threshold margin below 1e-12) and pairs of type-II items whose
skip length had a tie; both counts are reported."""
from __future__ import annotations

import numpy as np


def pair_keys(edges: np.ndarray) -> np.ndarray:
    e = np.asarray(edges, dtype=np.uint64).reshape(-1, 2)
    lo = np.minimum(e[:, 0], e[:, 1])
    hi = np.maximum(e[:, 0], e[:, 1])
    return (lo << np.uint64(32)) | hi


def compare(gpu_edges: np.ndarray, run, *, allow_extra: int = 0) -> dict:
    g = pair_keys(gpu_edges)
    o = pair_keys(run.edges)
    assert len(np.unique(g)) == len(g), "GPU output holds a pair twice"
    e = np.asarray(gpu_edges).reshape(-1, 2)
    assert np.all(e[:, 0] != e[:, 1]), "GPU output holds a self-loop"
    only_g = np.setdiff1d(g, o)
    only_o = np.setdiff1d(o, g)
    allowed = pair_keys(run.near) if len(run.near) else np.zeros(0, dtype=np.uint64)
    if len(run.ties):
        tp = np.array(sorted(run.tie_pairs()), dtype=np.uint64).reshape(-1, 2)
        allowed = np.union1d(allowed, pair_keys(tp))
    bad = np.setdiff1d(np.union1d(only_g, only_o), allowed)
    rep = {"gpu": len(g), "oracle": len(o), "only_gpu": len(only_g), "only_oracle": len(only_o),
           "near": len(run.near), "ties": len(run.ties), "unexplained": len(bad)}
    assert len(bad) <= allow_extra, f"edge sets differ outside the near-boundary pairs: {rep}"
    return rep
