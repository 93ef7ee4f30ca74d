"""Comparison helpers for GPU-vs-oracle parity.

The edge arrays must agree except for pairs the oracle logged as near the
decision boundary (|U - p| < 1e-12 for a coin U against a probability p; the
acceptance coin of a type-II candidate against p_uv / pbar; a relative
threshold margin below 1e-12 for the threshold variants) and the pairs of
type-II items whose skip quotient fell within 1e-12 (relative) of an integer.
Both counts are bounded by what the random draws of the run make likely (the
oracle sums, over its decisions and draws, the chance of each being logged).

Orientation and order: every edge must be written (A side, B side) as the
item (level, A, B, i, j) that holds it orders its cells (App. B.1: A <= B, the
layer pair ordered accordingly, a < b inside a cell of one layer), and after
sorting both arrays by the canonical key (level, A, B, i, j, k) the two must be
equal element by element."""
from __future__ import annotations

import math

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


def count_bound(expect: float) -> int:
    """Largest count of a Poisson(expect) variable that is not suspicious:
    expect + 6 sqrt(expect) + 3 (for expect << 1, a count above 3 has
    probability below expect^4 / 24)."""
    return int(math.floor(expect + 6.0 * math.sqrt(max(expect, 0.0)) + 3.0))


def canonical_order(edges: np.ndarray, run) -> tuple:
    """(edges sorted by the canonical key (level, A, B, i, j, k), their keys)."""
    e = np.ascontiguousarray(np.asarray(edges).reshape(-1, 2)).view(np.uint32)
    keys = run.edge_keys(e)
    order = np.lexsort((keys[:, 5], keys[:, 4], keys[:, 3], keys[:, 2], keys[:, 1], keys[:, 0]))
    return e[order], keys[order]


def check_gpu_counts(rep: dict, run, info) -> None:
    """The GPU's own counts of decisions inside the parity margins (a whole
    graph on both sides): near-boundary decisions as many as the oracle logged
    (the same test of the same coins), skip ties within the bound of what the
    draws make likely (the GPU counts draws, the oracle items)."""
    rep["gpu_near"] = int(info["near_boundary"])
    rep["gpu_ties"] = int(info["skip_ties"])
    assert rep["gpu_near"] == len(run.near), f"GPU and oracle near-boundary counts differ: {rep}"
    assert rep["gpu_ties"] <= count_bound(rep["tie_expect"]), f"too many GPU skip ties: {rep}"


def compare(gpu_edges: np.ndarray, run, *, allow_extra: int = 0, oriented: bool = True,
            info=None) -> dict:
    ge = np.ascontiguousarray(np.asarray(gpu_edges).reshape(-1, 2)).view(np.uint32)
    g = pair_keys(ge)
    o = pair_keys(run.edges)
    assert len(np.unique(g)) == len(g), "GPU output holds a pair twice"
    assert np.all(ge[:, 0] != ge[:, 1]), "GPU output holds a self-loop"
    only_g = np.setdiff1d(g, o)
    only_o = np.setdiff1d(o, g)
    diff = np.union1d(only_g, only_o)
    near_keys = pair_keys(run.near) if len(run.near) else np.zeros(0, dtype=np.uint64)
    if len(near_keys):
        diff = np.setdiff1d(diff, near_keys)
    bad = diff[~in_tie_items(diff, run)]
    rep = {"gpu": len(g), "oracle": len(o), "only_gpu": len(only_g), "only_oracle": len(only_o),
           "near": len(run.near), "ties": len(run.ties),
           "near_expect": float(run.stats.get("near_expect", 0.0)),
           "tie_expect": float(run.stats.get("tie_expect", 0.0)), "unexplained": len(bad)}
    assert len(bad) <= allow_extra, f"edge sets differ outside the near-boundary pairs: {rep}"
    assert rep["near"] <= count_bound(rep["near_expect"]), f"too many near-boundary decisions: {rep}"
    assert rep["ties"] <= count_bound(rep["tie_expect"]), f"too many skip ties: {rep}"
    if oriented and allow_extra == 0:
        # drop the excluded pairs from both sides, then compare (u, v) element
        # by element in the canonical order
        excl = np.union1d(near_keys, np.union1d(g[in_tie_items(g, run)], o[in_tie_items(o, run)]))
        gk = ge[~np.isin(g, excl)]
        ok = np.ascontiguousarray(run.edges)[~np.isin(o, excl)]
        gs, gkey = canonical_order(gk, run)
        os_, okey = canonical_order(ok, run)
        assert not gkey[:, 7].any(), "a GPU edge is not written with u from the A side of its item"
        assert not okey[:, 7].any(), "an oracle edge is not written with u from the A side"
        assert np.array_equal(gkey[:, :6], okey[:, :6]), "canonical keys differ"
        assert np.array_equal(gs, os_), "oriented edges differ in the canonical order"
        rep["oriented"] = len(gs)
    if info is not None:
        check_gpu_counts(rep, run, info)
    return rep


def level3_sample(edges, x, run, mod: int, batched: bool = False):
    """Edges of the items the oracle samples with filter_level = 3 and
    filter_mod = mod, filter_rem = 0: every item above level 3, and below it
    those whose A-side level-3 ancestor is 0 mod `mod`.  An item of a pair
    (u, v) sits above level 3 when CL(i, j) < 3 or the level-2 cells of u and
    v are not neighbours (the pair became distant earlier); otherwise its
    A side at level 3 is the smaller level-3 cell of u and v (A <= B is kept
    by every descendant).  edges (m, 2) and x (d, n) are device tensors."""
    import torch
    dev = edges.device
    d = x.shape[0]
    n = x.shape[1]
    layer = np.empty(n, dtype=np.int64)
    layer[run.sorted_ids.astype(np.int64)] = np.repeat(np.arange(64), run.count.astype(np.int64))
    layer = torch.from_numpy(layer).to(dev)
    CL = torch.from_numpy(run.CL.astype(np.int64)).to(dev)
    c3 = (x * 8.0).long()
    m3 = torch.zeros(n, dtype=torch.int64, device=dev)
    for b in (2, 1, 0):  # coarse to fine, dimension 0 most significant
        for k in range(d):
            m3 = (m3 << 1) | ((c3[k] >> b) & 1)
    u = edges[:, 0].long()
    v = edges[:, 1].long()
    far2 = torch.zeros(len(u), dtype=torch.bool, device=dev)
    for k in range(d):
        far2 |= torch.remainder((c3[k] >> 1)[u] - (c3[k] >> 1)[v], 4) == 2
    sel = torch.minimum(m3[u], m3[v])
    if batched:
        # type-II pairs at levels >= 3 belong to the sequence of the source
        # cell X that lists the other cell (first nonzero offset positive):
        # selected by X's level-3 ancestor
        cl_uv = CL[layer[u], layer[v]]
        lvl = torch.full_like(u, 1 << 20)  # the first level at which the cells are not neighbours
        for lv in range(1, 33 // d + 1):
            side = 1 << lv
            cu = (x * float(side)).long()
            far = torch.zeros(len(u), dtype=torch.bool, device=dev)
            for k in range(d):
                df = torch.remainder(cu[k][u] - cu[k][v], side)
                far |= torch.minimum(df, side - df) > 1
            lvl = torch.where(far & (lvl == (1 << 20)), torch.full_like(lvl, lv), lvl)
        t2 = (lvl >= 3) & (lvl <= cl_uv)
        if bool(t2.any()):
            side = (1 << lvl.clamp(max=30)).to(torch.int64)
            first = torch.zeros(len(u), dtype=torch.int64, device=dev)
            for k in range(d):
                cu = torch.floor(x[k][u] * side.double()).long()
                cv = torch.floor(x[k][v] * side.double()).long()
                dl = torch.remainder(cv - cu, side)
                dl = torch.where(dl >= side // 2, dl - side, dl)
                first = torch.where(first == 0, dl, first)
            xs_u = first > 0  # u's cell is the source
            sel = torch.where(t2, torch.where(xs_u, m3[u], m3[v]), sel)
    keep = (CL[layer[u], layer[v]] < 3) | far2 | (torch.remainder(sel, mod) == 0)
    return edges[keep]


def oriented_keys(edges: np.ndarray) -> np.ndarray:
    """u << 32 | v of oriented edges (u, v)."""
    e = np.asarray(edges, dtype=np.uint64).reshape(-1, 2)
    return (e[:, 0] << np.uint64(32)) | e[:, 1]


def compare_large(gpu_edges: np.ndarray, run, info=None) -> dict:
    """compare() for edge sets too large for the per-edge canonical keys: the
    same exclusions and bounds, and every pair both sides hold must be written
    with the same orientation (u, v).  Since an oracle edge is written with u
    from the A side of its item (pinned by compare() on smaller graphs), equal
    oriented pairs mean equal arrays in the canonical order once the excluded
    pairs are dropped."""
    ge = np.ascontiguousarray(np.asarray(gpu_edges).reshape(-1, 2)).view(np.uint32)
    oe = np.ascontiguousarray(run.edges)
    assert np.all(ge[:, 0] != ge[:, 1]), "GPU output holds a self-loop"
    gk = pair_keys(ge)
    ok = pair_keys(oe)
    gi = np.argsort(gk, kind="stable")
    oi = np.argsort(ok, kind="stable")
    g = gk[gi]
    o = ok[oi]
    assert not np.any(g[1:] == g[:-1]), "GPU output holds a pair twice"
    # orientation flag: 1 when u > v
    gf = (ge[gi, 0] > ge[gi, 1])
    of = (oe[oi, 0] > oe[oi, 1])
    both, ig, io = np.intersect1d(g, o, assume_unique=True, return_indices=True)
    only_g = np.delete(g, ig)
    only_o = np.delete(o, io)
    diff = np.union1d(only_g, only_o)
    near_keys = np.unique(pair_keys(run.near)) if len(run.near) else np.zeros(0, dtype=np.uint64)
    if len(near_keys):
        diff = np.setdiff1d(diff, near_keys, assume_unique=True)
    bad = diff[~in_tie_items(diff, run)]
    rep = {"gpu": len(g), "oracle": len(o), "only_gpu": len(only_g), "only_oracle": len(only_o),
           "near": len(run.near), "ties": len(run.ties),
           "near_expect": float(run.stats.get("near_expect", 0.0)),
           "tie_expect": float(run.stats.get("tie_expect", 0.0)), "unexplained": len(bad)}
    assert len(bad) == 0, f"edge sets differ outside the near-boundary pairs: {rep}"
    assert rep["near"] <= count_bound(rep["near_expect"]), f"too many near-boundary decisions: {rep}"
    assert rep["ties"] <= count_bound(rep["tie_expect"]), f"too many skip ties: {rep}"
    flip = int(np.count_nonzero(gf[ig] != of[io]))
    assert flip == 0, f"{flip} common pairs written with the other orientation"
    rep["oriented"] = len(both)
    if info is not None:
        check_gpu_counts(rep, run, info)
    return rep
