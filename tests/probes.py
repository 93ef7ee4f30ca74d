"""Builds and loads the GPU accuracy probe (tests/log2_probe.hip) with the
library's own compiler flags.  __graft_entry__.build() builds it beside the
library; the GPU tests only load what is built."""
from __future__ import annotations

import ctypes
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
OUT = os.path.join(HERE, "_build", "liblog2probe.so")


def build() -> str:
    from paper_1905_06706_amd import build as hb
    os.makedirs(os.path.dirname(OUT), exist_ok=True)
    tmp = OUT + f".tmp{os.getpid()}"
    cmd = [hb.hipcc(), *hb.FLAGS, "-I", hb.CSRC, "-o", tmp, os.path.join(HERE, "log2_probe.hip")]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError("hipcc failed:\n" + res.stdout + res.stderr)
    os.replace(tmp, OUT)
    return OUT


def load_log2() -> ctypes.CDLL:
    if not os.path.exists(OUT):
        raise RuntimeError(f"{OUT} is not built: run __graft_entry__.build() first")
    # bind to torch's HIP runtime (same soname), as the library does: a second
    # runtime in the process would hide the device from torch
    import torch  # noqa: F401
    lib = ctypes.CDLL(OUT)
    lib.log2_probe.argtypes = [ctypes.POINTER(ctypes.c_double)]
    lib.log2_probe.restype = ctypes.c_int
    return lib
