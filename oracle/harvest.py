"""FP64 oracle of the training-sample harvest (test infrastructure).

For a block X (n x k) with H X, Ritz values theta and converged eigenvectors
x* (n x nev) of the same matrix, column j yields one group:
    E_j  = x*_j - X (X^T x*_j)        the exact correction outside span(X)
    R_ij = (H X)_ij - theta_j X_ij,   U_ij = R_ij / s(d_i - sigma_j)
    (sigma_j the diagonal preconditioner's shift, theta_j unless an offset is given)
    p_i  = min(1, rows (1/(2n) + |E_ij| / (2 sum_l |E_lj|)))
and row i is kept when u(seed, group, i) < p_i, with weight 1/p_i.  The
uniform draw u is SplitMix64 (Steele, Lea & Flood, OOPSLA 2014): with
sm(x) the output for state x (add 0x9E3779B97F4A7C15, then the mix of the
published generator), u = (sm(sm(seed XOR sm(group)) + i) >> 11) 2^-53.
"""
from __future__ import annotations

import numpy as np

from .mlp import guard

_GOLDEN = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)


def splitmix64(x) -> np.ndarray:
    """One SplitMix64 output for each state x (uint64, wrapping arithmetic)."""
    with np.errstate(over="ignore"):
        z = np.asarray(x, dtype=np.uint64) + _GOLDEN
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
        return z ^ (z >> np.uint64(31))


def splitmix64_sequence(seed: int, count: int) -> np.ndarray:
    """The generator's first outputs from state `seed` (state advances by the golden gamma)."""
    with np.errstate(over="ignore"):
        states = np.uint64(seed) + _GOLDEN * np.arange(count, dtype=np.uint64)
    return splitmix64(states)


def uniform(seed: int, group: int, i) -> np.ndarray:
    h = splitmix64(np.uint64(seed) ^ splitmix64(np.uint64(group)))
    with np.errstate(over="ignore"):
        r = splitmix64(h + np.asarray(i, dtype=np.uint64))
    return (r >> np.uint64(11)).astype(np.float64) * 2.0 ** -53


def harvest_block(X, HX, theta, xstar, d, rownorm, tilemean, eps, rows, nev, seed, group0, offset=0.0):
    """Per column j < nev: dict of kept rows and their sample fields (in row order)."""
    X = np.asarray(X, dtype=np.float64)
    HX = np.asarray(HX, dtype=np.float64)
    xs = np.asarray(xstar, dtype=np.float64)
    theta = np.asarray(theta, dtype=np.float64)
    d = np.asarray(d, dtype=np.float64)
    n = X.shape[0]
    C = X.T @ xs
    out = []
    for j in range(nev):
        E = xs[:, j] - X @ C[:, j]
        tot = np.abs(E).sum()
        share = np.abs(E) / tot if tot > 0 else np.full(n, 1.0 / n)
        p = np.minimum(1.0, rows * (0.5 / n + 0.5 * share))
        u = uniform(seed, group0 + j, np.arange(n))
        keep = np.nonzero(u < p)[0]
        R = HX[:, j] - X[:, j] * theta[j]
        sigma_j = theta[j] - offset * (theta.max() - theta.min())
        U = R / guard(d - sigma_j, eps)
        out.append(dict(row=keep, p=p[keep], u=u[keep], p_all=p, u_all=u, E=E[keep], U=U[keep], w=1.0 / p[keep],
                        feat=np.stack([d[keep], np.full(keep.size, theta[j]), np.asarray(rownorm)[keep],
                                       np.asarray(tilemean)[keep]], axis=1),
                        Xrow=X[keep]))
    return out
