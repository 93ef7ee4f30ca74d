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


def in_tie_items(keys: np.ndarray, run) -> np.ndarray:
    """Mask of pair keys whose vertices lie in a logged tie item, on either
    side (items are ranges of sorted positions)."""
    keys = np.asarray(keys, dtype=np.uint64)
    inside = np.zeros(len(keys), dtype=bool)
    if len(keys) == 0 or len(run.ties) == 0:
        return inside
    pos = np.empty(len(run.sorted_ids), dtype=np.int64)
    pos[run.sorted_ids.astype(np.int64)] = np.arange(len(run.sorted_ids), dtype=np.int64)
    pu = pos[(keys >> np.uint64(32)).astype(np.int64)]
    pv = pos[(keys & np.uint64(0xFFFFFFFF)).astype(np.int64)]
    for a0, na, b0, nb in np.asarray(run.ties, dtype=np.int64):
        ina_u = (pu >= a0) & (pu < a0 + na)
        inb_v = (pv >= b0) & (pv < b0 + nb)
        ina_v = (pv >= a0) & (pv < a0 + na)
        inb_u = (pu >= b0) & (pu < b0 + nb)
        inside |= (ina_u & inb_v) | (ina_v & inb_u)
    return inside


def compare(gpu_edges: np.ndarray, run, *, allow_extra: int = 0) -> dict:
    g = pair_keys(gpu_edges)
    o = pair_keys(run.edges)
    assert len(np.unique(g)) == len(g), "GPU output holds a pair twice"
    e = np.asarray(gpu_edges).reshape(-1, 2)
    assert np.all(e[:, 0] != e[:, 1]), "GPU output holds a self-loop"
    only_g = np.setdiff1d(g, o)
    only_o = np.setdiff1d(o, g)
    diff = np.union1d(only_g, only_o)
    if len(run.near):
        diff = np.setdiff1d(diff, pair_keys(run.near))
    bad = diff[~in_tie_items(diff, run)]
    rep = {"gpu": len(g), "oracle": len(o), "only_gpu": len(only_g), "only_oracle": len(only_o),
           "near": len(run.near), "ties": len(run.ties), "unexplained": len(bad)}
    assert len(bad) <= allow_extra, f"edge sets differ outside the near-boundary pairs: {rep}"
    return rep
