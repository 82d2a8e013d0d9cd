"""Preconditioners of the LOBPCG step (test infrastructure): the diagonal
shift-inverse, and the block-diagonal preconditioner of shifted diagonal tiles
applied by FOM (further below).

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


# ---------------------------------------------------------------------------
# Block-diagonal preconditioner (Section 3.4): K = diag(K_1, ..., K_b), K_t the
# t-th diagonal tile of H shifted by sigma_j, each applied to the residual by
# m steps of the full orthogonalisation method (FOM; Saad, "Iterative Methods
# for Sparse Linear Systems", the method the paper cites): an Arnoldi process
# with modified Gram-Schmidt builds an orthonormal basis V_m of the Krylov
# space K_m(A, b) and the Hessenberg matrix H_m, and the approximate solution
# is x = V_m y with H_m y = ||b|| e_1.  Each column of R is its own right-hand
# side with its own shift (multiple Krylov spaces, Section 3.4).
# Each new Arnoldi vector is orthogonalised twice (two modified Gram-Schmidt
# passes, their coefficients summed into H_m; "twice is enough").  The paper
# does not fix the Gram-Schmidt variant; a single pass loses orthogonality
# completely on a shifted tile dominated by a constant diagonal (A = c I + E
# with |E| << c, the typical tile of a matrix with sorted diagonal): every
# A v_j is nearly parallel to v_j, and after a few steps V_m is no longer a
# basis, so the single-pass "FOM iterate" is rounding noise.

FOM_BREAKDOWN = 1e-12   # h_{j+1,j} <= this * ||A v_j||: K_j is invariant, x is exact
FOM_SINGULAR = 1e-12    # min |R_ii| <= this * max |h_ij| (H_m = QR, h over H_{m+1,m}): no FOM iterate


def diagonal_tiles(n: int, row_ptr, col, val, tile: int = 64) -> np.ndarray:
    """Dense symmetric diagonal tiles H[tT:(t+1)T, tT:(t+1)T] of H (given by
    its upper-triangle CSR), FP64, shape (ceil(n/T), T, T); rows past n get a
    unit diagonal (their right-hand sides are zero)."""
    nt = (n + tile - 1) // tile
    out = np.zeros((nt, tile, tile))
    rp = np.asarray(row_ptr, dtype=np.int64)
    ci = np.asarray(col, dtype=np.int64)
    v = np.asarray(val, dtype=np.float64)
    rows = np.repeat(np.arange(n, dtype=np.int64), np.diff(rp))
    same = (rows // tile) == (ci // tile)
    r, c, x = rows[same], ci[same], v[same]
    out[r // tile, r % tile, c % tile] = x
    out[r // tile, c % tile, r % tile] = x
    for i in range(n, nt * tile):
        out[i // tile, i % tile, i % tile] = 1.0
    return out


def fom(A: np.ndarray, b: np.ndarray, m: int, basis: bool = False):
    """m steps of FOM on A x = b from x = 0.  Returns (x, ok); ok is False when
    H_m is singular to working precision (then there is no FOM iterate).  With
    ``basis``, also the Arnoldi basis V_s and the square Hessenberg H_s of the
    s <= m steps taken (s < m after an invariant Krylov space)."""
    b = np.asarray(b, dtype=np.float64)
    beta = np.linalg.norm(b)
    if beta == 0.0:
        return (np.zeros_like(b), True) + ((np.zeros((b.size, 0)), np.zeros((0, 0))) if basis else ())
    N = b.size
    V = np.zeros((N, m + 1))
    Hm = np.zeros((m + 1, m))
    V[:, 0] = b / beta
    steps = m
    for j in range(m):
        w = A @ V[:, j]
        wnorm = np.linalg.norm(w)
        for _ in range(2):
            for i in range(j + 1):
                h = w @ V[:, i]
                Hm[i, j] += h
                w = w - h * V[:, i]
        Hm[j + 1, j] = np.linalg.norm(w)
        if Hm[j + 1, j] <= FOM_BREAKDOWN * wnorm:
            steps = j + 1
            break
        V[:, j + 1] = w / Hm[j + 1, j]
    Hs = Hm[:steps, :steps]
    extra = (V[:, :steps].copy(), Hs.copy()) if basis else ()
    rdiag = np.abs(np.diag(np.linalg.qr(Hs, mode="r")))
    if rdiag.min() <= FOM_SINGULAR * np.abs(Hm[:steps + 1, :steps]).max():
        return (np.zeros_like(b), False) + extra
    e1 = np.zeros(steps)
    e1[0] = beta
    y = np.linalg.solve(Hs, e1)
    return (V[:, :steps] @ y, True) + extra


def block_fom_precond(tiles: np.ndarray, R: np.ndarray, theta: np.ndarray, m: int, eps: float,
                      offset: float = 0.0) -> np.ndarray:
    """W = K^{-1} R with K_t = (diagonal tile t of H) - sigma_j I per column j,
    each block solved by m FOM steps; a block whose FOM has no iterate gets the
    diagonal step R_ij / s(d_i - sigma_j) instead.  `tiles` from diagonal_tiles."""
    R = np.asarray(R, dtype=np.float64)
    n, k = R.shape
    nt, T, _ = tiles.shape
    sig = shifts(theta, offset)
    W = np.zeros_like(R)
    for t in range(nt):
        lo, hi = t * T, min(n, (t + 1) * T)
        A0 = tiles[t]
        for j in range(k):
            b = np.zeros(T)
            b[:hi - lo] = R[lo:hi, j]
            x, ok = fom(A0 - sig[j] * np.eye(T), b, m)
            if ok:
                W[lo:hi, j] = x[:hi - lo]
            else:
                W[lo:hi, j] = R[lo:hi, j] / guard(np.diag(A0)[:hi - lo] - sig[j], eps)
    return W
