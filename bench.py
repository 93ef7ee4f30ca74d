"""Throughput benchmark of the gfx950 GIRG / HRG sampler.

python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME]

One step is one full call of the C ABI (points, constant, layers, sort, level
tables, prefix sums, enumeration, type-I tests, type-II geometric jumps, edge
compaction) for one graph of the workload; the inputs are synthetic and drawn
on the device from the seed.  Prints ONE JSON line on stdout; diagnostics go
to stderr.
"""
from __future__ import annotations

import argparse
import ctypes
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "edges/sec on 1 MI355X (+% HBM peak), mixed vs plain FP64, at oracle match"

# name: (description, generate kwargs).  Binomial GIRG workloads (and the
# batch) run two legs, plain FP64 and the FP32 filter with FP64 recheck; the
# others run FP64 only (the filter applies to binomial GIRGs).
WORKLOADS = {
    "girg_d3_n1e7": ("GIRG d=3 n=10^7 beta=2.3 T=0.8 avg_deg=20 seed=4",
                     dict(model=0, n=10**7, d=3, beta=2.3, T=0.8, avg_deg=20.0, seed=4)),
    "girg_d2_n2p20": ("GIRG d=2 n=2^20 beta=2.7 T=0.5 avg_deg=16 seed=2",
                      dict(model=0, n=2**20, d=2, beta=2.7, T=0.5, avg_deg=16.0, seed=2)),
    "hrg_n2p20": ("HRG n=2^20 alpha=0.75 T=0.5 avg_deg=10 (R solved) seed=3",
                  dict(model=1, n=2**20, d=1, alpha=0.75, T=0.5, avg_deg=10.0, seed=3)),
    "girg_d1_n1e4": ("GIRG d=1 n=10^4 beta=2.5 T=0 avg_deg=10 seed=1",
                     dict(model=0, n=10**4, d=1, beta=2.5, T=0.0, avg_deg=10.0, seed=1)),
    "girg_batch256": ("256 GIRGs, n=round(10^(3+3U)), d in {1,2}, beta~U[2.1,3], T in {0,0.3,0.9}, "
                      "avg_deg~U[8,32], seed 1000+b (numpy default_rng(5))",
                      dict(model=0, batch=256, master_seed=5)),
}
DEFAULT = "girg_d3_n1e7"
LEG_NAMES = {0: "fp64", 1: "mixed"}


def legs_of(wl: dict) -> list:
    """Precisions the workload runs: FP64, and the FP32 filter with FP64
    recheck where it applies (binomial GIRGs; the batch, whose threshold
    instances take the FP64 path either way)."""
    if "batch" in wl:
        return [0, 1]
    return [0, 1] if wl["model"] == 0 and wl["T"] > 0.0 else [0]


# Peak figures (MI355X): HBM3E 8 TB/s; VALU 256 CUs x 4 SIMD x 16 lanes x 2.4 GHz
HBM_PEAK_GBS = 8000.0
VALU_PEAK_TOPS = 256 * 4 * 16 * 2.4e9 / 1e12  # lane-operations per second, in T

# algorithmic VALU lane-operations per unit of work: the VALU instructions of
# each decision's arithmetic in the gfx950 build of the library's own device
# functions (d = 3; tests/test_opcount.py counts them in the assembly and
# keeps these figures within 10 % of the build)
OPS_TEST_T0 = 23.0      # threshold test: torus distance, r^d W <= kappa w_u w_v
OPS_TEST_BINOM = 175.0  # binomial test: distance, p_uv (FP64 log and exp series), half a Philox block, compare
OPS_DRAW = 149.0        # geometric draw: one Philox block, FP64 log series, skip quotient, end test
OPS_CAND = 140.0        # candidate: distance, p_uv, compare


# sources of the sampling kernels: HBM byte counters in profiles/ hold for
# the kernels built from sources with this hash only
KERNEL_SOURCES = ["paper_1905_06706_amd/csrc/sample.hip", "paper_1905_06706_amd/csrc/device_common.h",
                  "paper_1905_06706_amd/csrc/sampler.h", "paper_1905_06706_amd/csrc/fastpow.h"]
STAGE_KERNEL = {"type1": "k_type1<", "split1": "k_big1<", "type2": "k_type2<", "segments2": "k_heavy2<"}


def kernel_source_hash() -> str:
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def profiled_traffic(workload: str, stage: str):
    """HBM bytes per launch of the stage's kernel (FETCH_SIZE + WRITE_SIZE,
    each scaled by a plain copy's reading) from the committed rocprofv3
    summary, or None when there is none or the kernels changed since."""
    import re
    path = os.path.join(ROOT, "profiles", f"hbm_bytes_{workload}.txt")
    if not os.path.exists(path) or stage not in STAGE_KERNEL:
        return None
    want = kernel_source_hash()
    with open(path) as fh:
        for line in fh:
            m = re.match(r"traffic (.+) bytes_per_launch=(\d+) source_sha=(\w+)", line)
            if m and m.group(1).startswith(STAGE_KERNEL[stage]) and m.group(3) == want:
                return int(m.group(2))
    return None


def batch_params(hg, wl: dict, precision: int) -> list:
    """The batch recipe: per instance n = round(10^(3+3U)), d uniform in {1, 2},
    beta ~ U[2.1, 3.0], T uniform in {0, 0.3, 0.9}, average degree ~ U[8, 32],
    seed 1000 + b; parameters drawn from numpy's default_rng(master_seed)."""
    import numpy as np
    rng = np.random.default_rng(wl["master_seed"])
    out = []
    for b in range(wl["batch"]):
        n = int(round(10 ** (3 + 3 * rng.random())))
        d = int(rng.integers(1, 3))
        beta = float(rng.uniform(2.1, 3.0))
        T = float(rng.choice([0.0, 0.3, 0.9]))
        deg = float(rng.uniform(8.0, 32.0))
        out.append(hg.make_params(n, d, beta, T, deg, 0.0, 1000 + b, precision))
    return out


def make_call(hg, wl: dict, precision: int, type2_batch: int = 0):
    L = hg.load()
    if "batch" in wl:
        params = batch_params(hg, wl, precision)
        cnt = len(params)
        arr = (hg.Params * cnt)(*params)
        offs = (ctypes.c_uint64 * (cnt + 1))()
        infos = (hg.Info * cnt)()

        def call(buf, cap, m, info, stream):
            st = L.girg_generate_batch(arr, cnt, buf, cap, offs, infos, stream)
            m._obj.value = offs[cnt]
            # totals of the batch in `info`
            tot = {k: 0 for k in ("tests", "draws", "candidates", "rechecks", "type1_edges", "type2_edges",
                                  "near_boundary", "skip_ties")}
            for i in infos:
                for k in tot:
                    tot[k] += getattr(i, k)
            for k, v in tot.items():
                setattr(info._obj, k, v)
            info._obj.m = offs[cnt]
            call.ops = sum(i.tests * (OPS_TEST_T0 if p.T == 0.0 else OPS_TEST_BINOM)
                           + i.draws * OPS_DRAW + i.candidates * OPS_CAND for i, p in zip(infos, params))
            return st
        call.n_total = sum(p.n for p in params)
        call.params = params
        call.ops = 0.0
        return call
    if wl["model"] == 1:
        def call(buf, cap, m, info, stream):
            return L.girg_hrg(wl["n"], wl["alpha"], wl["T"], 0.0, wl["avg_deg"], wl["seed"], buf, cap,
                              m, info, stream)
        # the same graph as girg_generate parameters (R solved from the degree)
        call.params = hg.make_params(wl["n"], 1, 0.0, wl["T"], wl["avg_deg"], 0.0, wl["seed"], model=1,
                                     alpha=wl["alpha"])
        return call
    p = hg.make_params(wl["n"], wl["d"], wl["beta"], wl["T"], wl["avg_deg"], 0.0, wl["seed"], precision,
                       type2_batch=type2_batch)

    def call(buf, cap, m, info, stream):
        return L.girg_generate(ctypes.byref(p), buf, cap, m, info, stream)
    call.params = p
    return call


def cpu_info() -> dict:
    """Host cores and CPU model (the oracle runs single-threaded on them)."""
    model = ""
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        nproc = len(os.sched_getaffinity(0))
    except AttributeError:
        nproc = os.cpu_count() or 0
    return {"nproc": nproc, "cpu_model": model}


def oracle_check(hg, wl: dict, edges, info: dict, type2_batch: int = 0) -> tuple:
    """The oracle on the GPU's own points and constant (c, or R for the HRG),
    the same seed: the whole graph up to n = 2^21, above that every cell-pair
    item above level 3 plus the level-3 subtrees whose A-side ancestor is
    0 mod 512 (the GPU edges filtered the same way).  Returns the comparison
    report (edges that differ outside the near-boundary pairs and the tie
    items are 'unexplained') and the oracle's timing as the CPU baseline."""
    import numpy as np
    import torch
    import oracle
    from tests.parity import compare, level3_sample
    oracle.build()
    n = wl["n"]
    if wl["model"] == 1:
        R = info["R"]
        w, x = hg.points(n, model=1, alpha=wl["alpha"], R=R, seed=wl["seed"])
        kw = dict(T=wl["T"], model=1, R=R, alpha=wl["alpha"], seed=wl["seed"])
    else:
        w, x = hg.points(n, wl["d"], wl["beta"], seed=wl["seed"])
        kw = dict(T=wl["T"], c=info["c"], seed=wl["seed"], batch_type2=bool(type2_batch))
    sample = "the whole graph"
    if n > 2**21:
        kw.update(filter_level=3, filter_mod=512, filter_rem=0)
        sample = ("every cell-pair item above level 3 and the level-3 subtrees whose A-side "
                  "ancestor is 0 mod 512")
    wh = w.cpu().numpy()
    xh = np.ascontiguousarray(x.cpu().numpy().T)
    t0 = time.perf_counter()
    run = oracle.run(wh, xh, keep=True, **kw)
    dt = time.perf_counter() - t0
    m_orc = len(run.edges)
    if n > 2**21:
        edges = level3_sample(edges, x, run, 512, batched=bool(type2_batch))
    t1 = time.perf_counter()
    rep = {"sample": sample, "inputs": "the GPU's points and constant, same seed"}
    try:
        rep.update(compare(edges.cpu().numpy().view(np.uint32), run))
        rep["match"] = True
    except AssertionError as exc:
        rep["match"] = False
        rep["error"] = str(exc)[:400]
    rep["compare_s"] = time.perf_counter() - t1
    run.close()
    del w, x
    cpu = {"value": m_orc / dt, "unit": "edges/s", "cores": 1, "kind": "oracle",
           "sample": f"sampling of {sample} of the same graph (points and constant given): "
                     f"{m_orc} edges in {dt:.2f} s, single-threaded", **cpu_info()}
    return rep, cpu


def cpu_baseline_batch(params: list, budget_s: float = 15.0) -> dict:
    """The oracle, single-threaded, on the batch's instances in order (points,
    constant, sampling of each) until about `budget_s` seconds are spent."""
    import oracle
    oracle.build()
    t0 = time.perf_counter()
    m = 0
    k = 0
    for p in params:
        w, x = oracle.points_girg(p.n, p.d, p.beta, p.seed)
        c = oracle.solve_c(w, p.d, p.T, p.avg_deg)
        m += len(oracle.run(w, x, T=p.T, c=c, seed=p.seed).edges)
        k += 1
        if time.perf_counter() - t0 > budget_s:
            break
    dt = time.perf_counter() - t0
    return {"value": m / dt, "unit": "edges/s", "cores": 1, "kind": "oracle",
            "sample": f"the first {k} of {len(params)} instances, whole graphs; {m} edges in {dt:.2f} s",
            **cpu_info()}


def single_calls(hg, params: list, sp) -> dict:
    """The batch's instances through girg_generate one after another (the
    plain single-graph path, one call per instance, edges written): edges/s
    and ms, after one untimed pass, to set against the batched call."""
    import torch
    L = hg.load()
    m = ctypes.c_uint64(0)
    info = hg.Info()
    caps = []
    for p in params:
        st = L.girg_generate(ctypes.byref(p), None, 0, ctypes.byref(m), ctypes.byref(info), sp)
        if st not in (hg.GIRG_OK, hg.GIRG_EOVERFLOW):
            hg._check(st)
        caps.append(int(m.value))
    buf = torch.empty((max(max(caps), 1), 2), dtype=torch.int32, device="cuda")
    bp = ctypes.c_void_p(buf.data_ptr())
    total = 0
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for p, c in zip(params, caps):
        hg._check(L.girg_generate(ctypes.byref(p), bp, c, ctypes.byref(m), ctypes.byref(info), sp))
        total += m.value
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    return {"value": total / dt, "unit": "edges/s", "ms": dt * 1e3, "calls": len(params)}


# stage groups of the sweep, after the paper's breakdown of a run (Sec. 5.1)
SWEEP_GROUPS = {
    "points": ("points",),
    "constant": ("c_solve",),
    "pre": ("layer_key", "sort", "gather", "tables", "cells", "sources_count", "sources_fill"),
    "edges": ("type1", "type2", "deferred_prep", "split1", "segments2", "order"),
}


def sweep(steps: int, warmup: int) -> int:
    """Scaling sweep in the manner of the paper's Fig. 2: one parameter at a
    time around the base case d=1, n=2^15, T=0, beta=2.5, average degree 10
    (n up to 2^24, the degree, T, d), each graph counted but not stored (null
    edge buffer, capacity 0), as the paper measures.  Prints one JSON line
    with ms/step and ns/edge per stage group for every configuration."""
    import torch
    import paper_1905_06706_amd as hg
    L = hg.load()
    sp = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    base = dict(n=2**15, d=1, beta=2.5, T=0.0, deg=10.0)
    series = [("n", "n", [2**k for k in range(12, 25, 2)]),
              ("avg_deg", "deg", [5.0, 10.0, 20.0, 40.0, 80.0]),
              ("T", "T", [0.0, 0.1, 0.3, 0.5, 0.7, 0.9]),
              ("d", "d", [1, 2, 3, 4])]
    rows = []
    for name, key, values in series:
        for val in values:
            cfg = dict(base)
            cfg[key] = val
            if name != "n":
                cfg["n"] = 2**20
            p = hg.make_params(cfg["n"], cfg["d"], cfg["beta"], cfg["T"], cfg["deg"], 0.0, 7, 0)
            m = ctypes.c_uint64(0)
            for _ in range(warmup):
                L.girg_generate(ctypes.byref(p), None, 0, ctypes.byref(m), None, sp)
            # whole calls timed without stage events, then the same calls profiled
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(steps):
                st = L.girg_generate(ctypes.byref(p), None, 0, ctypes.byref(m), None, sp)
                if st not in (hg.GIRG_OK, hg.GIRG_EOVERFLOW):
                    hg._check(st)
            torch.cuda.synchronize()
            dt = (time.perf_counter() - t0) / steps
            hg.set_profiling(True)
            groups = {g: 0.0 for g in SWEEP_GROUPS}
            for _ in range(steps):
                L.girg_generate(ctypes.byref(p), None, 0, ctypes.byref(m), None, sp)
                for stage, ms in hg.stage_times():
                    for g, members in SWEEP_GROUPS.items():
                        if stage in members:
                            groups[g] += ms / steps
            torch.cuda.synchronize()
            hg.set_profiling(False)
            edges = max(int(m.value), 1)
            row = {"series": name, **cfg, "edges": int(m.value), "ms_per_step": dt * 1e3,
                   "ns_per_edge": dt * 1e9 / edges,
                   "ns_per_edge_by_stage": {g: v * 1e6 / edges for g, v in groups.items()}}
            rows.append(row)
            print(f"[sweep] {name}={val}: n={cfg['n']} m={m.value} {dt*1e3:.3f} ms "
                  f"{row['ns_per_edge']:.3f} ns/edge "
                  + " ".join(f"{g}={v:.3f}" for g, v in row["ns_per_edge_by_stage"].items()),
                  file=sys.stderr, flush=True)
    print(json.dumps({"sweep": rows, "steps": steps, "warmup": warmup, "data": "synthetic",
                      "mode": "count only (no edge store)"}), flush=True)
    return 0


def coupling(n: int = 10**6, deg: float = 100.0, alpha: float = 0.75, seed: int = 11) -> int:
    """The HRG / GIRG comparison of the paper's Sec. 5.3 (threshold variants),
    as one JSON line (see coupling_counts)."""
    t_start = time.perf_counter()
    out = coupling_counts(n, deg, alpha, seed)
    out.pop("_inputs", None)
    out["seconds"] = time.perf_counter() - t_start
    print(json.dumps(out), flush=True)
    return 0


def coupling_counts(n: int, deg: float, alpha: float = 0.75, seed: int = 11) -> dict:
    """An HRG (threshold) with average degree `deg` and the GIRG (threshold,
    d = 1) on the same points through the mapping of Sec. 2.3 (w =
    exp((R - r) / 2), x = angle / 2 pi).  Counts the edges the GIRG of
    expected degree `deg` lacks (HRG minus GIRG) and adds (GIRG minus HRG),
    the same for the GIRG whose expected degree is the HRG's realised one, the
    largest GIRG degree whose graph is a subgraph of the HRG (bisection; GIRG
    edge sets grow with c), and the smallest degree of a supergraph (from the
    largest c any HRG edge needs: r <= c w_u w_v / W).  `_inputs` holds the
    points and constants, for checks against the oracle."""
    import torch
    import paper_1905_06706_amd as hg
    R = hg.hrg_solve_R(n, alpha, 0.0, deg)
    r, x = hg.points(n, model=1, alpha=alpha, R=R, seed=seed)
    eh = hg.from_points(r, x, T=0.0, model=1, R=R, alpha=alpha, seed=seed).edges.long()

    def keys(e):
        lo = torch.minimum(e[:, 0], e[:, 1])
        hi = torch.maximum(e[:, 0], e[:, 1])
        return torch.sort(lo * (1 << 32) + hi).values

    kh = keys(eh)
    w = torch.exp((R - r) * 0.5).contiguous()
    W = float(w.sum())
    xg = x.contiguous()

    def girg_keys(avg_deg=0.0, c=0.0):
        res = hg.from_points(w, xg, T=0.0, c=c, avg_deg=avg_deg, seed=seed)
        return keys(res.edges.long()), res.info["c"]

    def count_not_in(a, b):
        """entries of sorted a that are not in sorted b"""
        if len(a) == 0:
            return 0
        if len(b) == 0:
            return len(a)
        i = torch.searchsorted(b, a).clamp(max=len(b) - 1)
        return int((b[i] != a).sum())

    kg, c_deg = girg_keys(avg_deg=deg)
    missing = count_not_in(kh, kg)
    additional = count_not_in(kg, kh)
    # largest degree with GIRG subset of HRG: bisection on the expected degree
    lo, hi = 0.01 * deg, deg
    c_sub = 0.0
    for _ in range(24):
        mid = (lo * hi) ** 0.5
        km, cm = girg_keys(avg_deg=mid)
        if count_not_in(km, kh) == 0:
            lo, c_sub = mid, cm
        else:
            hi = mid
    d_sub = lo
    # supergraph: the largest c needed by an HRG edge (d = 1 torus distance)
    u, v = eh[:, 0], eh[:, 1]
    df = (x[0, u] - x[0, v]).abs()
    dist = torch.minimum(df, 1.0 - df)
    c_super = float((dist * W / (w[u] * w[v])).max())
    D_super = hg.expected_degree(w.cpu().numpy(), 1, 0.0, c_super)
    d_hrg = 2.0 * len(kh) / n
    # the GIRG whose expected degree is the HRG's realised one
    km, cm = girg_keys(avg_deg=d_hrg)
    matched = {"girg_expected_degree": d_hrg, "girg_c": cm, "girg_edges": len(km),
               "missing_hrg_minus_girg": count_not_in(kh, km),
               "additional_girg_minus_hrg": count_not_in(km, kh)}
    return {"experiment": "HRG vs GIRG coupling (threshold variants)", "n": n, "alpha": alpha,
            "beta": 2 * alpha + 1, "R": R, "seed": seed, "hrg_edges": len(kh), "hrg_avg_degree": d_hrg,
            "girg_expected_degree": deg, "girg_c": c_deg, "girg_edges": len(kg),
            "missing_hrg_minus_girg": missing, "additional_girg_minus_hrg": additional,
            "subgraph_expected_degree": d_sub, "subgraph_c": c_sub, "supergraph_c": c_super,
            "supergraph_expected_degree": D_super, "at_hrg_degree": matched,
            "_inputs": {"r": r, "x": x, "w": w}}


def hbm_copy(mib: int, steps: int, warmup: int) -> int:
    """A plain device-to-device copy of a known size: the reference that
    scales the HBM byte counters (FETCH_SIZE, WRITE_SIZE) of the sampling
    kernels, and the achievable copy bandwidth."""
    import torch
    nbytes = mib << 20
    src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(warmup):
        dst.copy_(src)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        dst.copy_(src)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / max(steps, 1)
    print(json.dumps({"copy_bytes_read": nbytes, "copy_bytes_written": nbytes, "steps": steps,
                      "ms_per_copy": dt * 1e3, "GB_per_s": 2 * nbytes / dt / 1e9}), flush=True)
    return 0


def hbm_gather(mib: int, steps: int, warmup: int) -> int:
    """Reads 2^22 random 16-byte rows of a table of `mib` MiB (torch's
    index_select): beside the plain copy, the reference for what the HBM byte
    counters report for scattered 16-byte loads such as the sampling kernels'
    vertex records."""
    import torch
    rows = (mib << 20) // 16
    count = 1 << 22
    g = torch.Generator(device="cuda")
    g.manual_seed(7)
    table = torch.ones((rows, 4), dtype=torch.int32, device="cuda")
    idx = torch.randint(0, rows, (count,), device="cuda", generator=g)
    out = torch.empty((count, 4), dtype=torch.int32, device="cuda")
    for _ in range(warmup):
        torch.index_select(table, 0, idx, out=out)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        torch.index_select(table, 0, idx, out=out)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / max(steps, 1)
    print(json.dumps({"gather_rows": count, "row_bytes": 16, "table_bytes": rows * 16,
                      "index_bytes": count * 8, "bytes_written": count * 16, "steps": steps,
                      "ms_per_gather": dt * 1e3}), flush=True)
    return 0


def profiled_steps(hg, call, bp, cap, sp, nprof: int) -> tuple:
    """nprof calls with stage events, the concurrent sampling passes run one
    after another (profiling mode 2): every kernel's time is its own, as a
    kernel trace sees it.  Returns (mean stage times in ms, info of the last)."""
    import torch
    m = ctypes.c_uint64(0)
    info = hg.Info()
    hg.set_profiling(True, serial=True)
    acc: dict = {}
    try:
        for _ in range(nprof):
            hg._check(call(bp, cap, ctypes.byref(m), ctypes.byref(info), sp))
            for name, ms in hg.stage_times():
                acc[name] = acc.get(name, 0.0) + ms
        torch.cuda.synchronize()
    finally:
        hg.set_profiling(False)
    return {k: v / nprof for k, v in acc.items()}, info.as_dict()


def roofline(wl: dict, workload: str, stages: dict, info: dict) -> dict:
    """VALU roofline of the dominant sampling kernel, timed alone: its
    algorithmic lane-operations (units of work x VALU instructions per unit of
    the decision arithmetic) over its duration."""
    tb = OPS_TEST_T0 if wl["T"] == 0.0 else OPS_TEST_BINOM
    pw, pc = info["pass_work"], info["pass_cands"]
    per = {"type1": (pw[0] * tb, {"tests": pw[0]}),
           "split1": (pw[1] * tb, {"tests": pw[1]}),
           "type2": (pw[2] * OPS_DRAW + pc[2] * OPS_CAND, {"draws": pw[2], "candidates": pc[2]}),
           "segments2": (pw[3] * OPS_DRAW + pc[3] * OPS_CAND, {"draws": pw[3], "candidates": pc[3]})}
    ran = {k: stages[k] for k in per if stages.get(k, 0.0) > 0.0 and per[k][0] > 0}
    dom = max(ran, key=ran.get)
    ops, units = per[dom]
    ms = ran[dom]
    achieved = ops / (ms * 1e-3) / 1e12
    out = {"bound": "alu", "kernel": STAGE_KERNEL[dom] + "...>", "achieved": achieved,
           "peak": VALU_PEAK_TOPS, "unit": "Tlane-op/s", "frac": achieved / VALU_PEAK_TOPS,
           "traffic": profiled_traffic(workload, dom), "launch_ms": ms, "units_per_launch": units,
           "ops_per_unit": {"test": tb, "draw": OPS_DRAW, "candidate": OPS_CAND},
           "ops_per_launch": ops,
           "other_kernels": {STAGE_KERNEL[k] + "...>": {"ms": ran[k],
                                                        "frac": per[k][0] / (ran[k] * 1e-3) / 1e12 / VALU_PEAK_TOPS}
                             for k in ran if k != dom}}
    cnt = profiled_counters(workload, dom)
    if cnt:
        out["counters"] = cnt
    return out


def profiled_counters(workload: str, stage: str):
    """SQ counters of the stage's kernel from the committed rocprofv3 summary
    (VALU busy share, issued VALU lane-instructions per launch), or None when
    there is none or the kernels changed since."""
    import re
    path = os.path.join(ROOT, "profiles", f"sq_counters_{workload}.txt")
    if not os.path.exists(path) or stage not in STAGE_KERNEL:
        return None
    want = kernel_source_hash()
    with open(path) as fh:
        for line in fh:
            m = re.match(r"valu (.+) valu_busy=([\d.]+) valu_lane_ops_per_launch=(\d+) "
                         r"lanes_active=([\d.]+) source_sha=(\w+)", line)
            if m and m.group(1).startswith(STAGE_KERNEL[stage]) and m.group(5) == want:
                return {"valu_busy": float(m.group(2)), "valu_lane_ops_per_launch": int(m.group(3)),
                        "lanes_active": float(m.group(4)), "source": os.path.relpath(path, ROOT)}
    return None


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=30)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default=DEFAULT, choices=sorted(WORKLOADS))
    ap.add_argument("--precision", default="both", choices=["both", "fp64", "mixed"],
                    help="legs to run (default both where the FP32 filter applies)")
    ap.add_argument("--type2-batch", type=int, default=0, choices=[0, 1],
                    help="1: batched type-II jump sequences (GIRG d = 2, 3)")
    ap.add_argument("--no-cpu-baseline", action="store_true",
                    help="skip the oracle (both its timing and the oracle-match check)")
    ap.add_argument("--kernels-only", action="store_true",
                    help="only the profiled steps (passes one after another), for a kernel trace")
    ap.add_argument("--autotune", action="store_true",
                    help="autotune the launch shapes on this workload before the warm-up "
                         "(default: the library's tuning table)")
    ap.add_argument("--hbm-gather", type=int, default=0, metavar="MIB",
                    help="read 2^22 random 16-byte rows of a table of MIB MiB (counter reference)")
    ap.add_argument("--hbm-copy", type=int, default=0, metavar="MIB",
                    help="only time a plain device copy of MIB MiB (HBM calibration)")
    ap.add_argument("--sweep", action="store_true",
                    help="scaling sweep over n, degree, T and d (count only), one JSON line")
    ap.add_argument("--coupling", action="store_true",
                    help="HRG vs GIRG sub/supergraph experiment (threshold, n = 10^6), one JSON line")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (got --gpus {args.gpus}): the sampler has no "
              "multi-GPU path (DESIGN.md describes how it would shard)", file=sys.stderr)
        return 2
    if args.hbm_copy:
        return hbm_copy(args.hbm_copy, args.steps, args.warmup)
    if args.hbm_gather:
        return hbm_gather(args.hbm_gather, args.steps, args.warmup)
    if args.sweep:
        return sweep(min(args.steps, 5), min(args.warmup, 1))
    if args.coupling:
        return coupling()

    import torch
    import paper_1905_06706_amd as hg

    desc, wl = WORKLOADS[args.workload]
    hg.load()
    stream = torch.cuda.current_stream()
    sp = ctypes.c_void_p(stream.cuda_stream)
    legs = legs_of(wl)
    if args.precision != "both":
        want = 0 if args.precision == "fp64" else 1
        if want not in legs:
            print(f"[bench] {args.workload} has no {args.precision} leg", file=sys.stderr)
            return 2
        legs = [want]
    is_batch = "batch" in wl

    # per leg: the call, an output buffer sized by a first (counting) call
    # (for a kernel trace every call runs its passes one after another)
    if args.kernels_only:
        hg.set_profiling(True, serial=True)
    L = {}
    for q in legs:
        call = make_call(hg, wl, q, args.type2_batch)
        m = ctypes.c_uint64(0)
        info = hg.Info()
        st = call(None, 0, ctypes.byref(m), ctypes.byref(info), sp)
        if st not in (hg.GIRG_OK, hg.GIRG_EOVERFLOW):
            hg._check(st)
        cap = int(m.value)
        buf = torch.empty((max(cap, 1), 2), dtype=torch.int32, device="cuda")
        L[q] = dict(call=call, cap=cap, buf=buf, bp=ctypes.c_void_p(buf.data_ptr()))
    p0 = L[legs[0]]["call"].params
    # launch shapes (persistent grid size, batch workers): the library's table,
    # or tuned on this workload before the warm-up; they change no edge
    if not args.autotune:
        b, w = hg.tuning_get(p0[0] if is_batch else p0, batch=is_batch)
        tuning = {"autotuned": False, "blocks": b, **({"workers": w} if is_batch else {})}
    elif is_batch:
        b, w = hg.autotune_batch(p0, reps=1)
        tuning = {"autotuned": True, "blocks": b, "workers": w}
    else:
        tuning = {"autotuned": True, "blocks": hg.autotune(p0, reps=2)}
    print(f"[bench] tuning {tuning}", file=sys.stderr)

    if args.kernels_only:
        for q in legs:
            lg = L[q]
            stages, _ = profiled_steps(hg, lg["call"], lg["bp"], lg["cap"], sp, max(1, args.steps))
            print(json.dumps({"leg": LEG_NAMES[q], "workload": args.workload, "stages_ms": stages}), flush=True)
        return 0

    m = ctypes.c_uint64(0)
    info = hg.Info()
    for _ in range(args.warmup):
        for q in legs:
            lg = L[q]
            hg._check(lg["call"](lg["bp"], lg["cap"], ctypes.byref(m), ctypes.byref(info), sp))
    # timed: K steps per leg, each leg bracketed by device synchronisations
    # (no stage events); FP64 first, then the FP32 filter
    for q in legs:
        lg = L[q]
        edges = 0
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            hg._check(lg["call"](lg["bp"], lg["cap"], ctypes.byref(m), ctypes.byref(info), sp))
            edges += m.value
        torch.cuda.synchronize()
        lg["dt"] = time.perf_counter() - t0
        lg["edges"] = edges
        lg["m"] = int(m.value)
        lg["info"] = info.as_dict()
        print(f"[bench] {desc} {LEG_NAMES[q]}: m={m.value} steps={args.steps} "
              f"{lg['dt'] / args.steps * 1e3:.3f} ms/step", file=sys.stderr, flush=True)
    # kernel times, each pass alone (a few profiled steps after the timed ones)
    nprof = max(1, min(args.steps, 5))
    for q in legs:
        lg = L[q]
        lg["stages"], lg["pinfo"] = profiled_steps(hg, lg["call"], lg["bp"], lg["cap"], sp, nprof)
        for k, v in sorted(lg["stages"].items(), key=lambda kv: -kv[1]):
            print(f"[bench]   {LEG_NAMES[q]} {k:>14s} {v:9.4f} ms", file=sys.stderr)
    top = legs[-1]  # the reported leg: the FP32 filter where it runs
    lt = L[top]
    value = lt["edges"] / lt["dt"]
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "edges/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": lt["dt"] / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64" if top == 1 else "f64",
        "data": "synthetic",
        "config": {"workload": desc + (" (FP32 filter with FP64 recheck vs plain FP64)" if len(legs) > 1
                                       else " (FP64)"),
                   **{k: v for k, v in wl.items()}},
        "edges_per_step": lt["m"],
        "hbm_frac_edge_output": value * 8 / (HBM_PEAK_GBS * 1e9),
    }
    for q in legs:
        lg = L[q]
        out[LEG_NAMES[q]] = {"value": lg["edges"] / lg["dt"], "ms_per_step": lg["dt"] / args.steps * 1e3,
                             "edges_per_step": lg["m"], "near_boundary": lg["info"]["near_boundary"],
                             "skip_ties": lg["info"]["skip_ties"], "rechecks": lg["info"]["rechecks"]}
    if len(legs) > 1:
        out["mixed_vs_fp64"] = out["mixed"]["value"] / out["fp64"]["value"]
        same = L[0]["m"] == L[1]["m"] and torch.equal(L[0]["buf"][:L[0]["m"]], L[1]["buf"][:L[1]["m"]])
        out["mixed_equals_fp64"] = bool(same)
    if is_batch:
        ops = lt["call"].ops
        achieved = ops / (lt["dt"] / args.steps) / 1e12
        out["roofline"] = {"bound": "alu", "kernel": "whole batch step (all kernels, concurrent streams)",
                           "achieved": achieved, "peak": VALU_PEAK_TOPS, "unit": "Tlane-op/s",
                           "frac": achieved / VALU_PEAK_TOPS, "traffic": None,
                           "launch_ms": lt["dt"] / args.steps * 1e3, "ops_per_launch": ops}
    else:
        out["roofline"] = roofline(wl, args.workload + ("_mixed" if top == 1 else ""), lt["stages"],
                                   lt["pinfo"])
    out["stages_ms"] = lt["stages"]
    out["tuning"] = tuning
    if is_batch:
        out["single_calls"] = single_calls(hg, lt["call"].params, sp)
        print(f"[bench] single calls {out['single_calls']}", file=sys.stderr)
    if not args.no_cpu_baseline:
        if is_batch:
            out["cpu_baseline"] = cpu_baseline_batch(lt["call"].params)
        else:
            t0 = time.perf_counter()
            rep, cpu = oracle_check(hg, wl, lt["buf"][:lt["m"]], lt["info"], args.type2_batch)
            out["oracle_match"] = rep
            out["cpu_baseline"] = cpu
            print(f"[bench] oracle check ({time.perf_counter() - t0:.1f} s): {rep}", file=sys.stderr)
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
