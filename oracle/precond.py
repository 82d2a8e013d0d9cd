"""Diagonal shift-inverse preconditioner (test infrastructure).

The paper's preconditioner K is block diagonal, each block a diagonal tile of
H shifted by an approximation to one of the wanted eigenvalues (Section 3.4),
applied by a few FOM iterations.  With 1 x 1 tiles, FOM is exact after one
step and K^{-1} acts on column j of the residual as division by d_i - theta_j.
A guard keeps the divisor away from zero:
    s(x) = x                  if |x| >= eps
         = sign+(x) * eps     otherwise, with sign+(0) = +1.
Section 3.4 places the shift near an approximate wanted eigenvalue.  The
shift of column j is sigma_j = theta_j - c (theta_max - theta_min): c = 0 puts
it at the Ritz value itself; c > 0 keeps it c Ritz-value spreads below.
"""
from __future__ import annotations

import numpy as np


def guard(x: np.ndarray, eps: float) -> np.ndarray:
    x = np.asarray(x, dtype=np.float64)
    return np.where(np.abs(x) >= eps, x, np.where(x < 0, -eps, eps))


def shifts(theta: np.ndarray, offset: float = 0.0) -> np.ndarray:
    """sigma_j = theta_j - offset * (max theta - min theta)."""
    theta = np.asarray(theta, dtype=np.float64)
    return theta - offset * (theta.max() - theta.min())


def diag_precond(R: np.ndarray, d: np.ndarray, theta: np.ndarray, eps: float, offset: float = 0.0) -> np.ndarray:
    """W_ij = R_ij / s(d_i - sigma_j)."""
    R = np.asarray(R, dtype=np.float64)
    denom = guard(np.asarray(d, dtype=np.float64)[:, None] - shifts(theta, offset)[None, :], eps)
    return R / denom
