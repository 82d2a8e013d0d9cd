"""Named synthetic workloads, sized like the solver's target problems.

Each stands in for a nuclear CI Hamiltonian of the paper (Table 2): a
half-stored sparse symmetric matrix with a sorted diagonal, sought for its
lowest five eigenpairs with a block of k = 8 vectors (the paper's
experimental setting, Section 5).

    random_sym_20k    n = 20,000, 50 draws/row (~100 full nnz/row), FP64
    random_sym_1k     the same recipe at n = 1,000 (checked against dense eigh)
    tiled_2m          n = 2,000,000, 64x64 sparse tiles, ~0.3% tile density,
                      ~400 full nnz/row, FP32
    random_sym_10m    n = 10,000,000, 300 draws/row (~600 full nnz/row), FP32
    random_sym_2m     n = 2,000,000, 50 draws/row, FP32 (learned-preconditioner runs)
    zipf_50m          n = 50,000,000, power-law rows (Zipf 1.5, 20..20000), FP32
"""
from __future__ import annotations

import numpy as np

from . import random_sym, tiled, zipf, gaussian_block

WORKLOADS = {
    "random_sym_1k": dict(kind="random_sym", n=1000, draws=50, dmax=200.0, scale=0.5, f32=False, k=8),
    "random_sym_20k": dict(kind="random_sym", n=20000, draws=50, dmax=200.0, scale=0.5, f32=False, k=8),
    "tiled_2m": dict(kind="tiled", n=2_000_000, tile=64, tile_draws=47, p=400.0 / (64 * 95),
                     dmax=500.0, scale=0.1, f32=True, k=8),
    "random_sym_10m": dict(kind="random_sym", n=10_000_000, draws=300, dmax=200.0, scale=0.5,
                           f32=True, k=8),
    "random_sym_2m": dict(kind="random_sym", n=2_000_000, draws=50, dmax=200.0, scale=0.5,
                          f32=True, k=8),
    "zipf_50m": dict(kind="zipf", n=50_000_000, a=1.5, lmin=20, lmax=20000, dmax=1000.0,
                     scale=0.05, f32=True, k=16),
}


def make_matrix(name: str, seed: int = 0, n: int | None = None, f32: bool | None = None):
    w = dict(WORKLOADS[name])
    kind = w.pop("kind")
    w.pop("k")
    if n is not None:
        w["n"] = n
    if f32 is not None:
        w["f32"] = f32
    if kind == "random_sym":
        return random_sym(seed=seed, **w)
    if kind == "tiled":
        return tiled(seed=seed, **w)
    if kind == "zipf":
        return zipf(seed=seed, **w)
    raise KeyError(name)


def initial_block(n: int, k: int, seed: int = 1, dtype=np.float64) -> np.ndarray:
    """Gaussian starting block X0 (n x k, row-major)."""
    return gaussian_block(n, k, seed, dtype=dtype)
