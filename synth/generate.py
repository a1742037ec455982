"""Seeded generators for the five workloads.

The paper measures on matrix-factorisation vectors of four rating datasets
(Sec. 5.1) that are not available here; these generators stand in for them
with the shapes and norm spreads of such vectors: random directions, each
vector rescaled to a log-normal norm, optionally with users drawn from a
Gaussian mixture so that users share preferences.

Draw order is fixed: user directions, user norms, item directions, item
norms, then queries.  Generation is chunked by rows; numpy's Generator
produces the same stream whether a block is drawn at once or in pieces,
so the arrays do not depend on the chunk size.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Optional

import numpy as np

_CHUNK = 1 << 18  # rows per draw; bounds the FP64 temporaries


@dataclass(frozen=True)
class Config:
    name: str
    seed: int
    n: int
    m: int
    d: int
    k: int
    N: int
    user_sigma: float
    item_sigma: float
    user_clusters: int = 0        # 0 = isotropic directions
    cluster_std: float = 0.5
    n_queries: int = 0
    precision: str = "fp32"
    note: str = field(default="", compare=False)


CONFIGS = [
    Config("tiny", 0, 2_000, 1_000, 16, 10, 10, 0.3, 0.3,
           note="plain method, FP32"),
    Config("mf", 1, 100_000, 20_000, 50, 10, 10, 0.25, 0.6,
           note="matrix-factorisation shaped, FP32"),
    Config("bf16", 2, 500_000, 50_000, 100, 20, 50, 0.25, 0.8,
           user_clusters=64, cluster_std=0.5, precision="bf16",
           note="64-cluster users, BF16 screen"),
    Config("fp8", 3, 2_000_000, 100_000, 200, 10, 100, 0.25, 0.8,
           user_clusters=64, cluster_std=0.5, precision="fp8",
           note="64-cluster users, FP8 e4m3 screen"),
    Config("soft", 4, 1_000_000, 50_000, 100, 10, 0, 0.25, 0.8,
           user_clusters=64, cluster_std=0.5, n_queries=256,
           note="relaxed score over 256 query items"),
]


def _normalise_rows(x: np.ndarray) -> np.ndarray:
    nrm = np.sqrt(np.einsum("ij,ij->i", x, x))
    nrm[nrm == 0.0] = 1.0
    return x / nrm[:, None]


def isotropic(rng: np.random.Generator, count: int, d: int, sigma: float) -> np.ndarray:
    """N(0, I) directions, each row rescaled to a LogNormal(0, sigma) norm."""
    out = np.empty((count, d), dtype=np.float32)
    for s in range(0, count, _CHUNK):
        e = min(count, s + _CHUNK)
        out[s:e] = _normalise_rows(rng.standard_normal((e - s, d)))
    r = rng.lognormal(mean=0.0, sigma=sigma, size=count)
    for s in range(0, count, _CHUNK):
        e = min(count, s + _CHUNK)
        out[s:e] = (out[s:e].astype(np.float64) * r[s:e, None]).astype(np.float32)
    return out


def clustered(rng: np.random.Generator, count: int, d: int, sigma: float,
              n_clusters: int = 64, std: float = 0.5) -> np.ndarray:
    """Gaussian-mixture directions (n_clusters N(0, I) centres, isotropic
    spread `std`), each row rescaled to a LogNormal(0, sigma) norm."""
    centres = rng.standard_normal((n_clusters, d))
    z = rng.integers(0, n_clusters, size=count)
    out = np.empty((count, d), dtype=np.float32)
    for s in range(0, count, _CHUNK):
        e = min(count, s + _CHUNK)
        x = centres[z[s:e]] + std * rng.standard_normal((e - s, d))
        out[s:e] = _normalise_rows(x)
    r = rng.lognormal(mean=0.0, sigma=sigma, size=count)
    for s in range(0, count, _CHUNK):
        e = min(count, s + _CHUNK)
        out[s:e] = (out[s:e].astype(np.float64) * r[s:e, None]).astype(np.float32)
    return out


def make_config(cfg: Config | int, n: Optional[int] = None,
                m: Optional[int] = None):
    """Return (U, P) as C-contiguous FP32 arrays for a workload.

    `n`/`m` shrink the workload while keeping its distribution (the seed
    stream then differs from the full-size one)."""
    if isinstance(cfg, int):
        cfg = CONFIGS[cfg]
    n = cfg.n if n is None else n
    m = cfg.m if m is None else m
    rng = np.random.default_rng(cfg.seed)
    if cfg.user_clusters:
        U = clustered(rng, n, cfg.d, cfg.user_sigma, cfg.user_clusters, cfg.cluster_std)
    else:
        U = isotropic(rng, n, cfg.d, cfg.user_sigma)
    P = isotropic(rng, m, cfg.d, cfg.item_sigma)
    return np.ascontiguousarray(U), np.ascontiguousarray(P)


def make_queries(cfg: Config | int, count: Optional[int] = None,
                 seed_offset: int = 500) -> np.ndarray:
    """Query item vectors q ~ N(0, I/d), FP32, from their own stream."""
    if isinstance(cfg, int):
        cfg = CONFIGS[cfg]
    count = cfg.n_queries if count is None else count
    rng = np.random.default_rng(cfg.seed + seed_offset)
    q = rng.standard_normal((count, cfg.d)) / np.sqrt(cfg.d)
    return np.ascontiguousarray(q.astype(np.float32))


def subsample_users(cfg: Config | int, fraction: float = 0.01) -> np.ndarray:
    """Sorted seeded user subsample (indices) used where the full oracle
    is too slow."""
    if isinstance(cfg, int):
        cfg = CONFIGS[cfg]
    rng = np.random.default_rng(cfg.seed + 1000)
    cnt = max(1, int(cfg.n * fraction))
    return np.sort(rng.choice(cfg.n, cnt, replace=False)).astype(np.int64)
