"""Seeded synthetic inputs shared by the tests, the bench and smoke().

Holds none of the conversion arithmetic: only random coefficient vectors with
the decay profiles the paper uses for its experiments (Sec. 4: randn scaled so
that entry n is O(n^-p), p in {0, 0.5, 1, 1.5}), degree lists for mixed-degree
batches, and seeded output-row samples for large-N checks.
"""
from __future__ import annotations

import numpy as np


def rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def coeffs(N: int, p: float, seed: int, batch: int | None = None) -> np.ndarray:
    """alpha_k = z_k (k+1)^-p with z ~ N(0,1); shape (N+1,) or (batch, N+1), float64."""
    g = rng(seed)
    shape = (N + 1,) if batch is None else (batch, N + 1)
    z = g.standard_normal(shape)
    return z * (np.arange(N + 1, dtype=np.float64) + 1.0) ** (-float(p))


def batch_degrees(count: int, lo: int, hi: int, seed: int) -> np.ndarray:
    """Degrees log-uniform in [lo, hi] (floor of exp(U[ln lo, ln hi]))."""
    g = rng(seed)
    u = g.uniform(np.log(lo), np.log(hi), size=count)
    return np.clip(np.floor(np.exp(u)).astype(np.int64), lo, hi)


def sample_rows(N: int, count: int, seed: int) -> np.ndarray:
    """`count` seeded rows in [0, N] plus {0, 1, 2, N/2, N-1, N}, sorted, unique."""
    g = rng(seed)
    extra = np.array([0, 1, 2, N // 2, max(N - 1, 0), N], dtype=np.int64)
    r = np.concatenate([g.integers(0, N + 1, size=count, dtype=np.int64), extra])
    return np.unique(np.clip(r, 0, N))


def points(count: int, seed: int) -> np.ndarray:
    """Seeded evaluation points in [-1, 1]."""
    return rng(seed).uniform(-1.0, 1.0, size=count)
