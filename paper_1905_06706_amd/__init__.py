"""MI355X (gfx950) sampler for geometric inhomogeneous random graphs (GIRGs)
and hyperbolic random graphs (HRGs), after Blaesius et al., "Efficiently
Generating Geometric Inhomogeneous and Hyperbolic Random Graphs"
(arXiv:1905.06706).

This module is a thin ctypes binding of the C ABI declared in
``include/hipgirg.h``: it marshals arguments and uses PyTorch only to own
device memory and to name the current HIP stream.  Every step of the sampler
runs in the library's HIP kernels.  There is no fallback: if the built
library is missing, importing the bindings raises.
"""
from __future__ import annotations

import ctypes
import math
import os
from dataclasses import dataclass

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "_build", "libhipgirg.so")

GIRG_OK, GIRG_EINVAL, GIRG_ENOMEM, GIRG_EDEVICE, GIRG_EOVERFLOW, GIRG_ENOCONV = 0, -1, -2, -3, -4, -5
_STATUS = {-1: "EINVAL", -2: "ENOMEM", -3: "EDEVICE", -4: "EOVERFLOW", -5: "ENOCONV"}

EXPORTS = (
    "girg_generate", "girg_hrg", "girg_from_points", "girg_from_points_noalloc", "girg_points",
    "girg_solve_c",
    "girg_expected_degree", "hrg_solve_R", "hrg_expected_degree", "girg_generate_batch",
    "girg_release", "girg_last_error", "girg_version", "girg_set_profiling", "girg_stage_times",
    "girg_autotune", "girg_autotune_batch", "girg_tuning_get", "girg_tuning_set", "girg_tuning_save",
    "girg_tuning_load", "girg_tuning_reset",
)


class GirgError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{_STATUS.get(status, status)}: {msg}")
        self.status = status


class Params(ctypes.Structure):
    _fields_ = [
        ("n", ctypes.c_uint64), ("d", ctypes.c_int32), ("model", ctypes.c_int32),
        ("beta", ctypes.c_double), ("T", ctypes.c_double), ("avg_deg", ctypes.c_double),
        ("c", ctypes.c_double), ("alpha", ctypes.c_double), ("R", ctypes.c_double),
        ("seed", ctypes.c_uint64), ("precision", ctypes.c_int32), ("max_depth", ctypes.c_int32),
        ("cl_bias", ctypes.c_int32), ("type2_batch", ctypes.c_int32),
    ]


class Info(ctypes.Structure):
    _fields_ = [
        ("m", ctypes.c_uint64), ("type1_edges", ctypes.c_uint64), ("type2_edges", ctypes.c_uint64),
        ("tests", ctypes.c_uint64), ("draws", ctypes.c_uint64), ("candidates", ctypes.c_uint64),
        ("rechecks", ctypes.c_uint64), ("sources", ctypes.c_uint64),
        ("heavy_items", ctypes.c_uint64), ("split_items", ctypes.c_uint64),
        ("cells", ctypes.c_uint64), ("c", ctypes.c_double),
        ("W", ctypes.c_double), ("R", ctypes.c_double), ("L", ctypes.c_int32),
        ("D", ctypes.c_int32), ("reserved", ctypes.c_int32 * 2),
        ("pass_edges", ctypes.c_uint64 * 4), ("pass_work", ctypes.c_uint64 * 4),
        ("pass_cands", ctypes.c_uint64 * 4),
        ("near_boundary", ctypes.c_uint64), ("skip_ties", ctypes.c_uint64),
    ]

    def as_dict(self) -> dict:
        out = {}
        for k, _ in self._fields_:
            if k == "reserved":
                continue
            val = getattr(self, k)
            out[k] = list(val) if k.startswith("pass_") else val
        return out


_lib = None


def load() -> ctypes.CDLL:
    """Load the built library (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"HIP library not built: {LIB_PATH} (run paper_1905_06706_amd.build)")
    # torch ships its own HIP runtime under the same soname; importing it first
    # makes the library bind to that one, so the process holds a single
    # runtime (loading the library first mixes two and hides the device)
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    L = ctypes.CDLL(LIB_PATH)
    P, vp, u64, dbl = ctypes.POINTER, ctypes.c_void_p, ctypes.c_uint64, ctypes.c_double
    st = ctypes.c_int
    L.girg_generate.argtypes = [P(Params), vp, u64, P(u64), P(Info), vp]
    L.girg_hrg.argtypes = [u64, dbl, dbl, dbl, dbl, u64, vp, u64, P(u64), P(Info), vp]
    L.girg_from_points.argtypes = [P(Params), vp, vp, vp, u64, P(u64), P(Info), vp]
    L.girg_from_points_noalloc.argtypes = [P(Params), vp, vp, vp, u64, P(u64), P(Info), vp]
    L.girg_points.argtypes = [P(Params), vp, vp, vp]
    L.girg_solve_c.argtypes = [vp, u64, ctypes.c_int32, dbl, dbl, P(dbl)]
    L.girg_expected_degree.argtypes = [vp, u64, ctypes.c_int32, dbl, dbl, P(dbl)]
    L.hrg_solve_R.argtypes = [u64, dbl, dbl, dbl, P(dbl)]
    L.hrg_expected_degree.argtypes = [u64, dbl, dbl, dbl, P(dbl)]
    L.girg_generate_batch.argtypes = [P(Params), ctypes.c_int32, vp, u64, P(u64), P(Info), vp]
    L.girg_release.argtypes = []
    L.girg_set_profiling.argtypes = [ctypes.c_int32]
    L.girg_stage_times.argtypes = [P(dbl), P(ctypes.c_char_p), ctypes.c_int32]
    i32 = ctypes.c_int32
    L.girg_autotune.argtypes = [P(Params), i32, vp, P(i32)]
    L.girg_autotune_batch.argtypes = [P(Params), i32, i32, P(i32), P(i32)]
    L.girg_tuning_get.argtypes = [P(Params), i32, P(i32), P(i32)]
    L.girg_tuning_set.argtypes = [P(Params), i32, i32, i32]
    L.girg_tuning_save.argtypes = [ctypes.c_char_p]
    L.girg_tuning_load.argtypes = [ctypes.c_char_p]
    L.girg_tuning_reset.argtypes = []
    for name in EXPORTS:
        if name == "girg_stage_times":
            L.girg_stage_times.restype = ctypes.c_int32
        elif name in ("girg_last_error", "girg_version"):
            getattr(L, name).restype = ctypes.c_char_p
        else:
            getattr(L, name).restype = st
    _lib = L
    return L


def _check(status: int):
    if status != GIRG_OK:
        raise GirgError(status, load().girg_last_error().decode())


def version() -> str:
    return load().girg_version().decode()


def _stream(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def make_params(n, d=1, beta=2.5, T=0.0, avg_deg=0.0, c=0.0, seed=0, precision=0,
                max_depth=-1, cl_bias=0, model=0, alpha=0.0, R=0.0, type2_batch=0) -> Params:
    return Params(n=n, d=d, model=model, beta=beta, T=T, avg_deg=avg_deg, c=c, alpha=alpha,
                  R=R, seed=seed, precision=precision, max_depth=max_depth, cl_bias=cl_bias,
                  type2_batch=type2_batch)


def capacity_guess(n: int, avg_deg: float) -> int:
    m = n * avg_deg / 2.0
    return int(m * 1.3 + 6.0 * math.sqrt(max(m, 1.0)) + 4096)


@dataclass
class Result:
    edges: "object"   # torch.int32 tensor (m, 2) on the device, uint32 bit patterns
    info: dict


def _on(stream):
    """Allocations for work queued on `stream` are made on it, so that torch's
    caching allocator hands their memory to another stream only after it."""
    import contextlib
    import torch
    return contextlib.nullcontext() if stream is None else torch.cuda.stream(stream)


def _run_with_capacity(call, cap: int, device, stream=None):
    """call(edges_ptr, cap, m_ref, info_ref) -> status; grows the buffer once
    on overflow (the sampler is deterministic, so the rerun is identical)."""
    import torch
    for _ in range(2):
        with _on(stream):
            buf = torch.empty((max(cap, 1), 2), dtype=torch.int32, device=device)
        m = ctypes.c_uint64(0)
        info = Info()
        st = call(ctypes.c_void_p(buf.data_ptr()), cap, ctypes.byref(m), ctypes.byref(info))
        if st == GIRG_EOVERFLOW:
            cap = int(m.value)
            continue
        _check(st)
        return Result(buf[: m.value], info.as_dict())
    _check(GIRG_EOVERFLOW)


def generate(n: int, d: int = 1, beta: float = 2.5, T: float = 0.0, avg_deg: float = 0.0,
             c: float = 0.0, seed: int = 0, precision: int = 0, max_depth: int = -1,
             cl_bias: int = 0, cap: int | None = None, stream=None, device="cuda",
             type2_batch: int = 0) -> Result:
    """girg_generate: a GIRG with Pareto weights (w_min = 1) and uniform positions."""
    L = load()
    p = make_params(n, d, beta, T, avg_deg, c, seed, precision, max_depth, cl_bias,
                    type2_batch=type2_batch)
    if cap is None:
        cap = capacity_guess(n, avg_deg if avg_deg > 0 else 16.0)
    s = _stream(stream)
    return _run_with_capacity(lambda e, k, m, i: L.girg_generate(ctypes.byref(p), e, k, m, i, s),
                              cap, device, stream)


def hrg(n: int, alpha: float, T: float = 0.0, R: float = 0.0, avg_deg: float = 0.0,
        seed: int = 0, cap: int | None = None, stream=None, device="cuda") -> Result:
    """girg_hrg: a hyperbolic random graph through the GIRG mapping."""
    L = load()
    if cap is None:
        cap = capacity_guess(n, avg_deg if avg_deg > 0 else 16.0)
    s = _stream(stream)
    return _run_with_capacity(
        lambda e, k, m, i: L.girg_hrg(n, alpha, T, R, avg_deg, seed, e, k, m, i, s), cap, device,
        stream)


def from_points(w, x, T: float, c: float = 0.0, avg_deg: float = 0.0, seed: int = 0,
                model: int = 0, alpha: float = 0.0, R: float = 0.0, precision: int = 0,
                max_depth: int = -1, cl_bias: int = 0, cap: int | None = None,
                stream=None, type2_batch: int = 0) -> Result:
    """girg_from_points over device tensors: w (n,) float64, x (d, n) float64."""
    L = load()
    assert w.dtype.is_floating_point and w.element_size() == 8 and w.is_contiguous()
    assert x.element_size() == 8 and x.is_contiguous() and x.dim() == 2 and x.shape[1] == w.shape[0]
    n, d = int(w.shape[0]), int(x.shape[0])
    p = make_params(n, d, 0.0, T, avg_deg, c, seed, precision, max_depth, cl_bias, model, alpha, R,
                    type2_batch)
    if cap is None:
        cap = capacity_guess(n, avg_deg if avg_deg > 0 else 16.0)
    s = _stream(stream)
    wp, xp = ctypes.c_void_p(w.data_ptr()), ctypes.c_void_p(x.data_ptr())
    return _run_with_capacity(
        lambda e, k, m, i: L.girg_from_points(ctypes.byref(p), wp, xp, e, k, m, i, s), cap, w.device,
        stream)


def from_points_noalloc(w, x, edges, T: float, c: float = 0.0, seed: int = 0, model: int = 0,
                        alpha: float = 0.0, R: float = 0.0, precision: int = 0, max_depth: int = -1,
                        cl_bias: int = 0, stream=None, type2_batch: int = 0) -> tuple:
    """girg_from_points_noalloc into a caller-provided edge buffer `edges`
    (int32 (cap, 2) device tensor): returns (m, info); GirgError on overflow."""
    L = load()
    assert w.element_size() == 8 and w.is_contiguous()
    assert x.element_size() == 8 and x.is_contiguous() and x.dim() == 2 and x.shape[1] == w.shape[0]
    assert edges.dtype.itemsize == 4 and edges.is_contiguous() and edges.dim() == 2 and edges.shape[1] == 2
    n, d = int(w.shape[0]), int(x.shape[0])
    p = make_params(n, d, 0.0, T, 0.0, c, seed, precision, max_depth, cl_bias, model, alpha, R,
                    type2_batch)
    m = ctypes.c_uint64(0)
    info = Info()
    _check(L.girg_from_points_noalloc(ctypes.byref(p), ctypes.c_void_p(w.data_ptr()),
                                      ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(edges.data_ptr()),
                                      int(edges.shape[0]), ctypes.byref(m), ctypes.byref(info),
                                      _stream(stream)))
    return int(m.value), info.as_dict()


def points(n: int, d: int = 1, beta: float = 2.5, seed: int = 0, model: int = 0,
           alpha: float = 0.0, R: float = 0.0, stream=None, device="cuda"):
    """girg_points: (w, x) device tensors (x dimension-major, shape (d, n))."""
    import torch
    L = load()
    dd = 1 if model == 1 else d
    with _on(stream):
        w = torch.empty(n, dtype=torch.float64, device=device)
        x = torch.empty((dd, n), dtype=torch.float64, device=device)
    p = make_params(n, dd, beta, 0.0, 0.0, 0.0, seed, model=model, alpha=alpha, R=R)
    _check(L.girg_points(ctypes.byref(p), ctypes.c_void_p(w.data_ptr()),
                         ctypes.c_void_p(x.data_ptr()), _stream(stream)))
    return w, x


def solve_c(w_host, d: int, T: float, avg_deg: float) -> float:
    """girg_solve_c over host weights (numpy float64)."""
    import numpy as np
    w = np.ascontiguousarray(w_host, dtype=np.float64)
    out = ctypes.c_double(0.0)
    _check(load().girg_solve_c(ctypes.c_void_p(w.ctypes.data), len(w), d, T, avg_deg,
                               ctypes.byref(out)))
    return out.value


def expected_degree(w_host, d: int, T: float, c: float) -> float:
    import numpy as np
    w = np.ascontiguousarray(w_host, dtype=np.float64)
    out = ctypes.c_double(0.0)
    _check(load().girg_expected_degree(ctypes.c_void_p(w.ctypes.data), len(w), d, T, c,
                                       ctypes.byref(out)))
    return out.value


def hrg_solve_R(n: int, alpha: float, T: float, avg_deg: float) -> float:
    out = ctypes.c_double(0.0)
    _check(load().hrg_solve_R(n, alpha, T, avg_deg, ctypes.byref(out)))
    return out.value


def hrg_expected_degree(n: int, alpha: float, T: float, R: float) -> float:
    out = ctypes.c_double(0.0)
    _check(load().hrg_expected_degree(n, alpha, T, R, ctypes.byref(out)))
    return out.value


def generate_batch(params: list, cap: int | None = None, stream=None, device="cuda"):
    """girg_generate_batch: returns (edges (M, 2) int32 tensor, offsets list, infos)."""
    import torch
    L = load()
    cnt = len(params)
    arr = (Params * cnt)(*params)
    if cap is None:
        cap = sum(capacity_guess(p.n, p.avg_deg if p.avg_deg > 0 else 16.0) for p in params)
    s = _stream(stream)
    for _ in range(2):
        with _on(stream):
            buf = torch.empty((max(cap, 1), 2), dtype=torch.int32, device=device)
        offs = (ctypes.c_uint64 * (cnt + 1))()
        infos = (Info * cnt)()
        st = L.girg_generate_batch(arr, cnt, ctypes.c_void_p(buf.data_ptr()), cap, offs, infos, s)
        if st == GIRG_EOVERFLOW:
            cap = int(offs[cnt])
            continue
        _check(st)
        return buf[: offs[cnt]], list(offs), [i.as_dict() for i in infos]
    _check(GIRG_EOVERFLOW)


def autotune(params: Params, reps: int = 3, stream=None) -> int:
    """girg_autotune: the fastest persistent grid (workgroups) for params'
    workload class, now stored in the library's tuning table."""
    b = ctypes.c_int32(0)
    _check(load().girg_autotune(ctypes.byref(params), reps, _stream(stream), ctypes.byref(b)))
    return b.value


def autotune_batch(params: list, reps: int = 2) -> tuple:
    """girg_autotune_batch: (workgroups per instance, workers) of the fastest
    batch configuration, now stored in the tuning table."""
    cnt = len(params)
    arr = (Params * cnt)(*params)
    b, w = ctypes.c_int32(0), ctypes.c_int32(0)
    _check(load().girg_autotune_batch(arr, cnt, reps, ctypes.byref(b), ctypes.byref(w)))
    return b.value, w.value


def tuning_get(params: Params, batch: bool = False) -> tuple:
    """(workgroups, batch workers) that the next call with params would use."""
    b, w = ctypes.c_int32(0), ctypes.c_int32(0)
    _check(load().girg_tuning_get(ctypes.byref(params), 1 if batch else 0, ctypes.byref(b), ctypes.byref(w)))
    return b.value, w.value


def tuning_set(params: Params | None, blocks: int, batch: bool = False, workers: int = 0):
    p = ctypes.byref(params) if params is not None else None
    _check(load().girg_tuning_set(p, 1 if batch else 0, blocks, workers))


def tuning_save(path: str):
    _check(load().girg_tuning_save(os.fsencode(path)))


def tuning_load(path: str):
    _check(load().girg_tuning_load(os.fsencode(path)))


def tuning_reset():
    _check(load().girg_tuning_reset())


def set_profiling(on, serial: bool = False):
    """Stage timing on (True) or off; serial=True runs the otherwise
    concurrent sampling passes one after another (mode 2)."""
    _check(load().girg_set_profiling((2 if serial else 1) if on else 0))


def stage_times() -> list:
    """[(stage name, milliseconds)] of the last call (profiling on)."""
    L = load()
    ms = (ctypes.c_double * 64)()
    names = (ctypes.c_char_p * 64)()
    k = L.girg_stage_times(ms, names, 64)
    return [(names[i].decode(), ms[i]) for i in range(max(k, 0))]


def release():
    _check(load().girg_release())
