"""Whole-graph oracle runs split over processes (test infrastructure).

One run samples the cell pairs above a filter level (the subtrees below are
walked but pruned), the others sample the subtrees below it by the remainder
of their A-side ancestor at that level, skipping the pairs above.  Together
they sample every item exactly once, with the same coins as one plain run.
The workers are fresh interpreters (spawn) that import only numpy and the
oracle; the points reach them through .npy files."""
from __future__ import annotations

import multiprocessing as mp
import os
import shutil
import tempfile
from types import SimpleNamespace

import numpy as np


def _part(args):
    path, kw, part, nparts, level = args
    import oracle
    w = np.load(os.path.join(path, "w.npy"))
    x = np.load(os.path.join(path, "x.npy"))
    if part == 0:  # the top levels alone: no level-`level` ancestor has remainder 1 mod 1
        f = dict(filter_level=level, filter_mod=1, filter_rem=1)
    else:
        f = dict(filter_level=level, filter_mod=nparts, filter_rem=part - 1, filter_skip_top=True)
    run = oracle.run(w, x, keep=False, **kw, **f)
    out = dict(edges=run.edges, near=run.near, ties=run.ties,
               stats={k: run.stats[k] for k in ("near_expect", "tie_expect", "tests", "draws",
                                                  "candidates", "near", "ties")})
    if part == 0:
        out["sorted_ids"] = run.sorted_ids
        out["L"], out["D"], out["W"] = run.stats["L"], run.stats["D"], run.stats["W"]
    return out


def workers() -> int:
    try:
        ncpu = len(os.sched_getaffinity(0))
    except AttributeError:
        ncpu = os.cpu_count() or 1
    return max(1, min(16, ncpu))


def run_whole(w: np.ndarray, x: np.ndarray, *, level: int = 3, nparts: int = 32,
              nproc: int | None = None, **kw) -> SimpleNamespace:
    """The oracle's whole graph over points (w, x) with run() keywords kw,
    from 1 + nparts runs on nproc processes.  Returns a Run-like namespace:
    edges, near, ties, sorted_ids, stats (summed)."""
    tmp = tempfile.mkdtemp(prefix="orcpool")
    try:
        np.save(os.path.join(tmp, "w.npy"), np.ascontiguousarray(w, dtype=np.float64))
        np.save(os.path.join(tmp, "x.npy"), np.ascontiguousarray(x, dtype=np.float64))
        tasks = [(tmp, kw, p, nparts, level) for p in range(nparts + 1)]
        with mp.get_context("spawn").Pool(nproc or workers()) as pool:
            parts = pool.map(_part, tasks, chunksize=1)
    finally:
        shutil.rmtree(tmp, ignore_errors=True)
    stats: dict = {}
    for p in parts:
        for k, v in p["stats"].items():
            stats[k] = stats.get(k, 0.0) + v
    stats.update(L=parts[0]["L"], D=parts[0]["D"], W=parts[0]["W"])
    return SimpleNamespace(
        edges=np.concatenate([p["edges"] for p in parts]).reshape(-1, 2),
        near=np.concatenate([p["near"] for p in parts]).reshape(-1, 2),
        ties=np.concatenate([p["ties"] for p in parts]).reshape(-1, 4),
        sorted_ids=parts[0]["sorted_ids"], stats=stats)
