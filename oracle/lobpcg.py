"""LOBPCG in FP64, following the paper's Algorithm 1 step by step
(test infrastructure; see the package docstring).

Algorithm 1 (Section 2):
    [C, Theta] = RayleighRitz(H, X0);  X = X0 C;  R = H X - X Theta;  P = empty
    for i = 1..maxiter:
        W = K^{-1} R
        S = [X, W, P];  [C, Theta] = RayleighRitz(H, S)          (eq. rreig)
        X = S C                                                  (eq. xupd)
        R = H X - X Theta
        P = W C_2 + P C_3                                        (eq. pupd)
        count converged columns by their relative residual norms; exit when done
    H X and H P are carried by the recurrences eqs. upd1-upd2, so H W is the
    only sparse product per iteration.

Readings where the paper is silent (each is shared by the HIP path):
  * relative residual:  rel_j = ||r_j|| / (max(|theta_j|, tau) ||x_j||),
    tau = 1e-3 * gamma, gamma = max_i sum_j |H_ij| (Gershgorin bound);
  * only the nev wanted columns are counted; on apparent convergence H X is
    recomputed by an explicit product, theta_j = x_j^T H x_j, and the test is
    repeated (guards the drift of the eqs. upd1-upd2 recurrences);
  * W is orthogonalised against X (W <- W - X (X^T W)) and then put through
    Cholesky QR (Section 3.5); if the Cholesky factor fails, the Gram matrix
    is scaled to unit diagonal and shifted by 1e-12 (shifted Cholesky QR),
    and only if that fails too the solve stops with "not SPD";
  * P and H P are scaled column-wise by 1/||P_j|| after each update;
  * if O = S^T S is not positive definite, P is dropped for that iteration;
  * the preconditioner is the diagonal shift-inverse (oracle.precond) unless a
    callable is supplied.
Options for the FP32-robustness row (Section 3.5; eqs. upd1-upd2 drift):
  * cholqr_passes=2: every Cholesky QR of W is CholeskyQR2 (a second pass on
    its result);
  * soft_lock=True: a column whose relative residual was at or below tol at
    the last check is locked: its residual direction W_j and its P_j leave
    the search space (S = [X, W_active, P_active]) while X_j stays in the
    Rayleigh-Ritz basis, so converged columns stop feeding noise into W and
    P; a locked column is released when its residual rises above tol again.
Status codes match the library: 0 OK, -4 not SPD, -5 not converged.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Callable, Optional

import numpy as np
from threadpoolctl import threadpool_limits

from . import SymMatrix
from .dense import NotSPD, assemble_pencil, cholqr, cholqr2, gram, rayleigh_ritz
from .precond import diag_precond

OK, ENOTSPD, ENOCONV = 0, -4, -5


@dataclass
class Result:
    theta: np.ndarray                 # nev Ritz values (ascending)
    X: np.ndarray                     # n x nev Ritz vectors
    iters: int
    status: int
    rel: np.ndarray                   # final relative residuals of all k columns
    theta_all: np.ndarray             # all k Ritz values
    X_all: np.ndarray                 # n x k block
    n_spmm: int = 0
    theta_hist: list = field(default_factory=list)
    rel_hist: list = field(default_factory=list)
    resid_hist: list = field(default_factory=list)
    p_dropped: int = 0
    cholqr_shifts: int = 0
    cholqr_retries: int = 0          # Cholesky QRs retried after projecting W again
    active_hist: list = field(default_factory=list)   # active (unlocked) columns per iteration


def rel_residuals(R: np.ndarray, X: np.ndarray, theta: np.ndarray, tau: float) -> np.ndarray:
    rn = np.linalg.norm(R, axis=0)
    xn = np.linalg.norm(X, axis=0)
    return rn / (np.maximum(np.abs(theta), tau) * xn)


def lobpcg(H: SymMatrix, X0: np.ndarray, nev: int, tol: float = 1e-6, maxiter: int = 5000,
           precond: Optional[Callable] = "diag", d: Optional[np.ndarray] = None,
           tau_rel: float = 1e-3, eps_rel: float = 1e-5,
           callback: Optional[Callable] = None, precond_offset: float = 0.0, cholqr_passes: int = 1,
           soft_lock: bool = False) -> Result:
    """See :func:`_lobpcg`.  Small problems run the dense BLAS single-threaded
    (thread start-up dominates there); the arithmetic is unchanged."""
    args = (H, X0, nev, tol, maxiter, precond, d, tau_rel, eps_rel, callback, precond_offset, cholqr_passes,
            soft_lock)
    if X0.shape[0] < 200_000:
        with threadpool_limits(1, user_api="blas"):
            return _lobpcg(*args)
    return _lobpcg(*args)


def _lobpcg(H: SymMatrix, X0: np.ndarray, nev: int, tol: float = 1e-6, maxiter: int = 5000,
            precond: Optional[Callable] = "diag", d: Optional[np.ndarray] = None,
            tau_rel: float = 1e-3, eps_rel: float = 1e-5,
            callback: Optional[Callable] = None, precond_offset: float = 0.0, cholqr_passes: int = 1,
            soft_lock: bool = False) -> Result:
    """Lowest ``nev`` eigenpairs of H from the starting block X0 (n x k, k >= nev).

    ``precond``: "diag" (needs ``d``, the diagonal of H; its shift lies
    ``precond_offset`` Ritz-value spreads below theta_j), None (identity), or a
    callable ``f(R, theta, X) -> W``.  ``callback(it, X, R, theta, W)`` is called
    each iteration before the Rayleigh-Ritz step (used to harvest training data).
    """
    X0 = np.asarray(X0, dtype=np.float64)
    n, k = X0.shape
    if not (1 <= nev <= k and 3 * k <= n):
        raise ValueError("need 1 <= nev <= k and 3k <= n")
    if cholqr_passes not in (1, 2):
        raise ValueError("cholqr_passes must be 1 or 2")
    qr = cholqr2 if cholqr_passes == 2 else cholqr
    gamma = H.gershgorin()
    tau = tau_rel * gamma
    eps = eps_rel * gamma
    if precond == "diag":
        if d is None:
            raise ValueError("diag preconditioner needs d")
        dd = np.asarray(d, dtype=np.float64)

        def apply_k(R, theta, X):
            return diag_precond(R, dd, theta, eps, precond_offset)
    elif precond is None:
        def apply_k(R, theta, X):
            return R.copy()
    else:
        apply_k = precond

    n_spmm = 0
    # Algorithm 1, start: Rayleigh-Ritz on X0
    HX0 = H @ X0
    n_spmm += 1
    G, O = assemble_pencil([X0], [HX0])
    theta, C = rayleigh_ritz(G, O, k)
    X = X0 @ C
    HX = HX0 @ C
    R = HX - X * theta
    P = HP = None
    res = Result(theta=theta[:nev], X=X[:, :nev], iters=0, status=ENOCONV, rel=None,
                 theta_all=theta, X_all=X)
    p_dropped = 0
    it = 0
    while True:
        rel = rel_residuals(R, X, theta, tau)
        if np.all(rel[:nev] <= tol):
            # confirm with an explicit product (guards recurrence drift)
            HX = H @ X
            n_spmm += 1
            theta = np.einsum("ij,ij->j", X, HX) / np.einsum("ij,ij->j", X, X)
            R = HX - X * theta
            rel = rel_residuals(R, X, theta, tau)
            if np.all(rel[:nev] <= tol):
                res.status = OK
                break
        if it >= maxiter:
            break
        it += 1
        # soft locking: the columns converged at this check leave W and P
        active = rel > tol if soft_lock else np.ones(k, dtype=bool)
        res.active_hist.append(int(active.sum()))
        # preconditioned residual W = K^{-1} R
        W = np.asarray(apply_k(R, theta, X), dtype=np.float64)[:, active]
        if P is not None:
            P, HP = P[:, active], HP[:, active]
            if P.shape[1] == 0:
                P = HP = None
        if callback is not None:
            callback(it, X, R, theta, W)
        if W.shape[1] == 0:
            # every column locked (possible only with soft_lock before the
            # confirmation): the basis cannot grow, stop as not converged
            break
        # orthogonalise against X, then Cholesky QR (Section 3.5); a shifted
        # Cholesky QR is the fallback when W^T W is numerically singular
        # (if the shifted one fails too, W is projected once more and both are
        # tried again before giving up)
        W = W - X @ gram(X, W)
        orthonormal = False
        for attempt in range(2):
            try:
                W, _ = qr(W)
                orthonormal = True
            except NotSPD:
                try:
                    W, _ = qr(W, shift=1e-12)
                    res.cholqr_shifts += 1
                    orthonormal = True
                except NotSPD:
                    res.cholqr_retries += attempt == 0
                    W = W - X @ gram(X, W)
            if orthonormal:
                break
        if not orthonormal:
            res.status = ENOTSPD
            break
        HW = H @ W
        n_spmm += 1
        # Rayleigh-Ritz on S = [X, W, P] (eq. rreig)
        if P is not None:
            S, HS = [X, W, P], [HX, HW, HP]
        else:
            S, HS = [X, W], [HX, HW]
        try:
            G, O = assemble_pencil(S, HS)
            theta, C = rayleigh_ritz(G, O, k)
        except NotSPD:
            if P is None:
                res.status = ENOTSPD
                break
            p_dropped += 1
            S, HS = [X, W], [HX, HW]
            try:
                G, O = assemble_pencil(S, HS)
                theta, C = rayleigh_ritz(G, O, k)
            except NotSPD:
                res.status = ENOTSPD
                break
        # update of X, P and their products with the recurrences eqs. upd1-upd2
        Sm = np.hstack(S)
        HSm = np.hstack(HS)
        X = Sm @ C
        HX = HSm @ C
        P = Sm[:, k:] @ C[k:]
        HP = HSm[:, k:] @ C[k:]
        pn = np.linalg.norm(P, axis=0)
        scale = np.where(pn > 0, 1.0 / np.where(pn > 0, pn, 1.0), 1.0)
        P = P * scale
        HP = HP * scale
        R = HX - X * theta
        res.theta_hist.append(theta.copy())
        res.resid_hist.append(np.linalg.norm(R, axis=0))
        res.rel_hist.append(rel_residuals(R, X, theta, tau))
    res.theta = theta[:nev].copy()
    res.theta_all = theta.copy()
    res.X = X[:, :nev].copy()
    res.X_all = X
    res.iters = it
    res.rel = rel_residuals(R, X, theta, tau)
    res.n_spmm = n_spmm
    res.p_dropped = p_dropped
    return res
