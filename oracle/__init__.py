"""Python access to the plain C oracle (``oracle.c``).

TEST INFRASTRUCTURE.  Only ``tests/``, the smoke check and the
``cpu_baseline`` leg of ``bench.py`` may import this package.  It shares no
code with the HIP library (``paper_1905_06706_amd``) and never imports it.

The oracle is a sequential FP64 implementation of the GIRG sampler of
Blaesius et al. (arXiv:1905.06706): weights and positions (Sec. 2), weight
buckets, comparison and insertion levels (Sec. 3.1), Morton-sorted cells with
prefix sums (Sec. 3.4, Lemma 1), Algorithm 1 (Sec. 3.3) with the double
counting rules of App. B.1, and the estimation of c (App. B.2).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB_DIR = os.path.join(_HERE, "_build")
_LIB = os.path.join(_LIB_DIR, "liboracle.so")

MAX_LAYERS = 64
NSTATS = 24
STAT_NAMES = {
    0: "W", 1: "w0", 2: "L", 3: "D", 4: "Dmax", 5: "nb_pairs", 6: "dist_pairs",
    7: "type1_items", 8: "type2_items", 9: "tests", 10: "draws", 11: "candidates",
    12: "edges", 13: "near", 14: "ties", 15: "segments", 16: "kappa_or_coshR",
    17: "type1_edges", 18: "type2_edges", 19: "near_expect", 20: "tie_expect", 21: "seqs",
}


def build(force: bool = False) -> str:
    """Compile ``oracle.c`` with gcc into ``_build/liboracle.so``."""
    os.makedirs(_LIB_DIR, exist_ok=True)
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + f".tmp{os.getpid()}"
        subprocess.check_call([
            "gcc", "-O2", "-std=c11", "-Wall", "-Wextra", "-ffp-contract=off",
            "-fno-fast-math", "-fPIC", "-shared", "-o", tmp, _SRC, "-lm",
        ])
        os.replace(tmp, _LIB)
    return _LIB


class _Params(ctypes.Structure):
    _fields_ = [
        ("n", ctypes.c_uint64), ("d", ctypes.c_int32), ("model", ctypes.c_int32),
        ("T", ctypes.c_double), ("c", ctypes.c_double), ("alpha", ctypes.c_double),
        ("R", ctypes.c_double), ("seed", ctypes.c_uint64), ("max_depth", ctypes.c_int32),
        ("cl_bias", ctypes.c_int32), ("accept_all", ctypes.c_int32),
        ("filter_level", ctypes.c_int32), ("filter_mod", ctypes.c_uint32),
        ("filter_rem", ctypes.c_uint32), ("filter_skip_top", ctypes.c_int32),
        ("batch_type2", ctypes.c_int32),
    ]


_lib = None


def build_variant(src_text: str, out_path: str) -> str:
    """Compile an edited copy of the oracle's source (the mutation tests plant
    mistakes in such copies to show that the pins catch them) with the same
    flags into out_path."""
    src = out_path + ".c"
    with open(src, "w") as fh:
        fh.write(src_text)
    subprocess.check_call([
        "gcc", "-O2", "-std=c11", "-w", "-ffp-contract=off", "-fno-fast-math", "-fPIC",
        "-shared", "-I", _HERE, "-o", out_path, src, "-lm",
    ])
    return out_path


class use_library:
    """Context manager: every function of this module calls the library at
    `path` (a variant from build_variant) until the block ends."""

    def __init__(self, path: str):
        self.path = path

    def __enter__(self):
        global _lib
        self.saved = _lib
        _lib = None
        _lib = _load(self.path)
        return self

    def __exit__(self, *exc):
        global _lib
        _lib = self.saved
        return False


def lib() -> ctypes.CDLL:
    global _lib
    if _lib is None:
        _lib = _load(_LIB if os.path.exists(_LIB) else build())
    return _lib


def _load(path: str) -> ctypes.CDLL:
    L = ctypes.CDLL(path)
    P = ctypes.POINTER
    u32p, u64p, dblp = P(ctypes.c_uint32), P(ctypes.c_uint64), P(ctypes.c_double)
    L.orc_philox4x32_10.argtypes = [u32p, u32p, u32p]
    L.orc_u53.restype = ctypes.c_double
    L.orc_u53.argtypes = [ctypes.c_uint32, ctypes.c_uint32]
    L.orc_u53_open.restype = ctypes.c_double
    L.orc_u53_open.argtypes = [ctypes.c_uint32, ctypes.c_uint32]
    L.orc_morton_encode.restype = ctypes.c_uint64
    L.orc_morton_encode.argtypes = [u32p, ctypes.c_int, ctypes.c_int]
    L.orc_morton_decode.argtypes = [ctypes.c_uint64, ctypes.c_int, ctypes.c_int, u32p]
    L.orc_points_girg.argtypes = [ctypes.c_uint64, ctypes.c_int, ctypes.c_double,
                                  ctypes.c_uint64, dblp, dblp]
    L.orc_points_hrg.argtypes = [ctypes.c_uint64, ctypes.c_double, ctypes.c_double,
                                 ctypes.c_uint64, dblp, dblp]
    L.orc_expected_avg_degree.restype = ctypes.c_double
    L.orc_expected_avg_degree.argtypes = [ctypes.c_uint64, ctypes.c_int, ctypes.c_double,
                                          ctypes.c_double, dblp]
    L.orc_solve_c.restype = ctypes.c_int
    L.orc_solve_c.argtypes = [ctypes.c_uint64, ctypes.c_int, ctypes.c_double,
                              ctypes.c_double, dblp, dblp]
    L.orc_hrg_expected_avg_degree.restype = ctypes.c_double
    L.orc_hrg_expected_avg_degree.argtypes = [ctypes.c_uint64, ctypes.c_double,
                                              ctypes.c_double, ctypes.c_double]
    L.orc_hrg_solve_R.restype = ctypes.c_int
    L.orc_hrg_solve_R.argtypes = [ctypes.c_uint64, ctypes.c_double, ctypes.c_double,
                                  ctypes.c_double, dblp]
    L.orc_run_graph.restype = ctypes.c_void_p
    L.orc_run_graph.argtypes = [P(_Params), dblp, dblp]
    L.orc_last_error.restype = ctypes.c_char_p
    L.orc_free.argtypes = [ctypes.c_void_p]
    for name in ("orc_num_edges", "orc_num_near", "orc_num_ties"):
        getattr(L, name).restype = ctypes.c_uint64
        getattr(L, name).argtypes = [ctypes.c_void_p]
    L.orc_copy_edges.argtypes = [ctypes.c_void_p, u32p]
    L.orc_copy_near.argtypes = [ctypes.c_void_p, u32p]
    L.orc_copy_ties.argtypes = [ctypes.c_void_p, u64p]
    L.orc_copy_sorted_ids.argtypes = [ctypes.c_void_p, u32p]
    L.orc_stats.argtypes = [ctypes.c_void_p, dblp]
    L.orc_tables.argtypes = [ctypes.c_void_p, P(ctypes.c_int32), P(ctypes.c_int32),
                             P(ctypes.c_int64), dblp]
    L.orc_pair_item.argtypes = [ctypes.c_void_p, ctypes.c_uint32, ctypes.c_uint32,
                                P(ctypes.c_int64)]
    L.orc_level_counts.argtypes = [ctypes.c_void_p, u64p, u64p]
    L.orc_edge_keys.argtypes = [ctypes.c_void_p, u32p, ctypes.c_uint64, P(ctypes.c_int64)]
    return L


def _ptr(a: np.ndarray, ctype):
    return a.ctypes.data_as(ctypes.POINTER(ctype))


# ---- random-number contract -------------------------------------------------
def philox4x32_10(ctr, key) -> np.ndarray:
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    out = np.zeros(4, dtype=np.uint32)
    lib().orc_philox4x32_10(_ptr(c, ctypes.c_uint32), _ptr(k, ctypes.c_uint32),
                            _ptr(out, ctypes.c_uint32))
    return out


def u53(lo: int, hi: int) -> float:
    return lib().orc_u53(lo, hi)


def u53_open(lo: int, hi: int) -> float:
    return lib().orc_u53_open(lo, hi)


def morton_encode(coords, d: int, bits: int) -> int:
    c = np.ascontiguousarray(coords, dtype=np.uint32)
    return int(lib().orc_morton_encode(_ptr(c, ctypes.c_uint32), d, bits))


def morton_decode(code: int, d: int, bits: int) -> np.ndarray:
    out = np.zeros(d, dtype=np.uint32)
    lib().orc_morton_decode(code, d, bits, _ptr(out, ctypes.c_uint32))
    return out


# ---- points ----------------------------------------------------------------
def points_girg(n: int, d: int, beta: float, seed: int):
    w = np.empty(n, dtype=np.float64)
    x = np.empty((n, d), dtype=np.float64)
    lib().orc_points_girg(n, d, beta, seed, _ptr(w, ctypes.c_double), _ptr(x, ctypes.c_double))
    return w, x


def points_hrg(n: int, alpha: float, R: float, seed: int):
    r = np.empty(n, dtype=np.float64)
    x = np.empty((n, 1), dtype=np.float64)
    lib().orc_points_hrg(n, alpha, R, seed, _ptr(r, ctypes.c_double), _ptr(x, ctypes.c_double))
    return r, x


# ---- parameter estimation --------------------------------------------------
def expected_avg_degree(w: np.ndarray, d: int, T: float, c: float) -> float:
    w = np.ascontiguousarray(w, dtype=np.float64)
    return lib().orc_expected_avg_degree(len(w), d, T, c, _ptr(w, ctypes.c_double))


def solve_c(w: np.ndarray, d: int, T: float, avg_deg: float) -> float:
    w = np.ascontiguousarray(w, dtype=np.float64)
    out = ctypes.c_double(0.0)
    rc = lib().orc_solve_c(len(w), d, T, avg_deg, _ptr(w, ctypes.c_double), ctypes.byref(out))
    if rc != 0:
        raise RuntimeError(lib().orc_last_error().decode())
    return out.value


def hrg_expected_avg_degree(n: int, alpha: float, T: float, R: float) -> float:
    return lib().orc_hrg_expected_avg_degree(n, alpha, T, R)


def hrg_solve_R(n: int, alpha: float, T: float, avg_deg: float) -> float:
    out = ctypes.c_double(0.0)
    rc = lib().orc_hrg_solve_R(n, alpha, T, avg_deg, ctypes.byref(out))
    if rc != 0:
        raise RuntimeError(lib().orc_last_error().decode())
    return out.value


# ---- sampling --------------------------------------------------------------
@dataclass
class Run:
    edges: np.ndarray          # (m, 2) uint32, original ids, oracle order
    near: np.ndarray           # (k, 2) uint32 near-boundary pairs
    ties: np.ndarray           # (t, 4) uint64 a0, Na, b0, Nb in sorted positions
    sorted_ids: np.ndarray     # (n,) uint32
    stats: dict
    CL: np.ndarray             # (64, 64) int32
    I: np.ndarray              # (64,) int32
    count: np.ndarray          # (64,) int64
    ext: np.ndarray            # (64,) float64
    level_nb: np.ndarray
    level_dist: np.ndarray
    _handle: int = field(default=0, repr=False)

    def tie_pairs(self) -> set:
        """All vertex pairs of items whose skip sequence had a tie."""
        out = set()
        for a0, na, b0, nb in self.ties:
            for a in range(int(a0), int(a0 + na)):
                for b in range(int(b0), int(b0 + nb)):
                    u, v = int(self.sorted_ids[a]), int(self.sorted_ids[b])
                    out.add((min(u, v), max(u, v)))
        return out

    def pair_items(self, pairs: np.ndarray) -> np.ndarray:
        """Classify vertex pairs (u, v): level, A, B, i, j, type, swapped."""
        out = np.zeros((len(pairs), 7), dtype=np.int64)
        buf = (ctypes.c_int64 * 7)()
        L = lib()
        for k, (u, v) in enumerate(pairs):
            L.orc_pair_item(self._handle, int(u), int(v), buf)
            out[k] = np.frombuffer(buf, dtype=np.int64)
        return out

    def edge_keys(self, edges: np.ndarray) -> np.ndarray:
        """(m, 8) int64 per edge (u, v): level, A, B, i, j, k, type and a
        flag set when the edge is not written with u from the A side."""
        e = np.ascontiguousarray(np.asarray(edges).reshape(-1, 2).view(np.uint32)
                                 if np.asarray(edges).dtype != np.uint32
                                 else np.asarray(edges).reshape(-1, 2))
        out = np.zeros((len(e), 8), dtype=np.int64)
        if len(e):
            assert self._handle, "run(..., keep=True) is needed for edge keys"
            lib().orc_edge_keys(self._handle, _ptr(e, ctypes.c_uint32), len(e), _ptr(out, ctypes.c_int64))
        return out

    def close(self):
        if self._handle:
            lib().orc_free(self._handle)
            self._handle = 0

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def run(w: np.ndarray, x: np.ndarray, *, T: float, c: float = 0.0, seed: int = 0,
        model: int = 0, alpha: float = 0.0, R: float = 0.0, max_depth: int = -1,
        cl_bias: int = 0, accept_all: bool = False, filter_level: int = 0,
        filter_mod: int = 0, filter_rem: int = 0, filter_skip_top: bool = False,
        batch_type2: bool = False, keep: bool = False) -> Run:
    """Sample one graph over the given points (GIRG: weights w, HRG: radii w)."""
    w = np.ascontiguousarray(w, dtype=np.float64)
    x = np.ascontiguousarray(x, dtype=np.float64)
    if x.ndim == 1:
        x = x.reshape(-1, 1)
    n, d = x.shape
    assert len(w) == n
    p = _Params(n=n, d=d, model=model, T=T, c=c, alpha=alpha, R=R, seed=seed,
                max_depth=max_depth, cl_bias=cl_bias, accept_all=int(accept_all),
                filter_level=filter_level, filter_mod=filter_mod, filter_rem=filter_rem,
                filter_skip_top=int(filter_skip_top), batch_type2=int(batch_type2))
    L = lib()
    h = L.orc_run_graph(ctypes.byref(p), _ptr(w, ctypes.c_double), _ptr(x, ctypes.c_double))
    if not h:
        raise ValueError(L.orc_last_error().decode())
    m = L.orc_num_edges(h)
    edges = np.zeros((m, 2), dtype=np.uint32)
    if m:
        L.orc_copy_edges(h, _ptr(edges, ctypes.c_uint32))
    k = L.orc_num_near(h)
    near = np.zeros((k, 2), dtype=np.uint32)
    if k:
        L.orc_copy_near(h, _ptr(near, ctypes.c_uint32))
    t = L.orc_num_ties(h)
    ties = np.zeros((t, 4), dtype=np.uint64)
    if t:
        L.orc_copy_ties(h, _ptr(ties, ctypes.c_uint64))
    sid = np.zeros(n, dtype=np.uint32)
    L.orc_copy_sorted_ids(h, _ptr(sid, ctypes.c_uint32))
    st = np.zeros(NSTATS, dtype=np.float64)
    L.orc_stats(h, _ptr(st, ctypes.c_double))
    CL = np.zeros((MAX_LAYERS, MAX_LAYERS), dtype=np.int32)
    I = np.zeros(MAX_LAYERS, dtype=np.int32)
    cnt = np.zeros(MAX_LAYERS, dtype=np.int64)
    ext = np.zeros(MAX_LAYERS, dtype=np.float64)
    L.orc_tables(h, _ptr(CL, ctypes.c_int32), _ptr(I, ctypes.c_int32),
                 _ptr(cnt, ctypes.c_int64), _ptr(ext, ctypes.c_double))
    lnb = np.zeros(40, dtype=np.uint64)
    ldist = np.zeros(40, dtype=np.uint64)
    L.orc_level_counts(h, _ptr(lnb, ctypes.c_uint64), _ptr(ldist, ctypes.c_uint64))
    stats = {name: st[i] for i, name in STAT_NAMES.items()}
    r = Run(edges, near, ties, sid, stats, CL, I, cnt, ext, lnb, ldist, _handle=h)
    if not keep:
        r.close()
    return r
