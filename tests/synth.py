"""Seeded synthetic inputs shared by the oracle tests and the GPU parity tests.

This module holds none of the sampler's arithmetic: it only draws arrays of
weights, positions and radii with numpy's own generator, in the shapes and
distributions of the paper's workloads (Pareto weights with w_min = 1,
positions uniform on the torus as multiples of 2^-53, HRG radii), so that both
implementations can be fed bit-identical inputs.
"""
from __future__ import annotations

import numpy as np


def rng(seed: int) -> np.random.Generator:
    return np.random.default_rng(seed)


def positions(n: int, d: int, seed: int) -> np.ndarray:
    """(n, d) uniform positions in [0,1), exact multiples of 2^-53."""
    g = rng(seed)
    q = g.integers(0, 2**53, size=(n, d), dtype=np.int64)
    return q.astype(np.float64) * 2.0**-53


def pareto_weights(n: int, beta: float, seed: int) -> np.ndarray:
    """(n,) weights with P(w > t) = t^{-(beta-1)}, w >= 1."""
    g = rng(seed + 7919)
    return (1.0 - g.random(n)) ** (-1.0 / (beta - 1.0))


def hrg_radii(n: int, alpha: float, R: float, seed: int) -> np.ndarray:
    """(n,) radii in [0, R] with density alpha sinh(alpha r) / (cosh(alpha R) - 1)."""
    g = rng(seed + 104729)
    u = g.random(n)
    r = np.arccosh(1.0 + u * (np.cosh(alpha * R) - 1.0)) / alpha
    return np.minimum(r, R)


def clustered_positions(n: int, d: int, seed: int, clusters: int = 4) -> np.ndarray:
    """Positions concentrated in a few tiny boxes (adversarial cell occupancy)."""
    g = rng(seed + 31)
    centres = g.random((clusters, d))
    idx = g.integers(0, clusters, size=n)
    jitter = g.random((n, d)) * 2.0**-12
    x = np.mod(centres[idx] + jitter, 1.0)
    q = np.floor(x * 2.0**53).astype(np.int64)
    q = np.minimum(q, 2**53 - 1)
    return q.astype(np.float64) * 2.0**-53


def seam_positions(n: int, d: int, seed: int, width: float = 2.0**-7) -> np.ndarray:
    """Positions within `width` of the torus seam 0 = 1 in every coordinate,
    half just above 0 and half just below 1 (exact multiples of 2^-53), so
    that most close pairs are close only across the seam."""
    g = rng(seed + 1013)
    q = g.integers(0, int(width * 2**53), size=(n, d), dtype=np.int64)
    hi = g.random((n, d)) < 0.5
    q = np.where(hi, 2**53 - 1 - q, q)
    return q.astype(np.float64) * 2.0**-53
