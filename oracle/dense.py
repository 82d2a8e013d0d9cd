"""FP64 dense steps of LOBPCG (test infrastructure; see the package docstring).

Cholesky QR (paper Section 3.5):  B = W^T W,  B = R^T R,  W <- W R^{-1};
CholeskyQR2 repeats it once on the result.
Gram blocks (eq. Glower): only the lower blocks of G = S^T H S and
O = S^T S are formed; each upper block is the transpose of its lower
counterpart, and each diagonal block is averaged with its own transpose.
Rayleigh-Ritz (eq. rreig): the pencil (G, O), scaled to a unit diagonal of O,
is reduced with the Cholesky factor of O and solved by a symmetric
eigensolver; the k leftmost Ritz pairs are kept, in ascending order (the paper
calls LAPACK dsygv, which does the same reduction).  O counts as not positive
definite (the caller then drops P) when that Cholesky factor has a squared
pivot at or below RR_PIVOT_TOL: a basis that nearly lost a direction passes a
plain Cholesky but the reduced pencil then yields Ritz values outside the
spectrum.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla


class NotSPD(np.linalg.LinAlgError):
    pass


# smallest squared pivot accepted in the Cholesky of the unit-diagonal-scaled O
RR_PIVOT_TOL = 1e-7


def gram(A: np.ndarray, B: np.ndarray) -> np.ndarray:
    """A^T B in FP64 (inputs upcast exactly)."""
    return np.asarray(A, dtype=np.float64).T @ np.asarray(B, dtype=np.float64)


def cholesky_upper(B: np.ndarray) -> np.ndarray:
    """R upper triangular with B = R^T R; raises NotSPD if B is not positive definite."""
    try:
        L = np.linalg.cholesky(B)
    except np.linalg.LinAlgError as e:
        raise NotSPD(str(e)) from None
    if not np.all(np.isfinite(L)) or np.any(np.diag(L) <= 0):
        raise NotSPD("non-positive pivot")
    return L.T.copy()


def cholqr(W: np.ndarray, shift: float | None = None) -> tuple[np.ndarray, np.ndarray]:
    """Cholesky QR: returns (W R^{-1}, R).  Raises NotSPD when W^T W is not SPD.

    With ``shift``, the Gram matrix is first scaled to unit diagonal,
    B' = S B S with S = diag(B)^{-1/2}, and B' + shift*I is factored (shifted
    Cholesky QR, Fukaya et al. 2020); then R = R' S^{-1}.
    """
    B = gram(W, W)
    B = 0.5 * (B + B.T)
    if shift is None:
        R = cholesky_upper(B)
    else:
        dg = np.diag(B)
        if np.any(dg <= 0):
            raise NotSPD("zero column")
        s = 1.0 / np.sqrt(dg)
        Rp = cholesky_upper(B * np.outer(s, s) + shift * np.eye(B.shape[0]))
        R = Rp / s[None, :]
    Q = sla.solve_triangular(R, np.asarray(W, dtype=np.float64).T, trans="T", lower=False).T
    return Q, R


def cholqr2(W: np.ndarray, shift: float | None = None) -> tuple[np.ndarray, np.ndarray]:
    """CholeskyQR2 (Fukaya, Nakatsukasa, Yanagisawa, Yamamoto 2014): Cholesky QR
    applied twice, W = Q (R2 R1).  The first pass (shifted when ``shift`` is
    given) leaves Q1 with orthogonality error of order eps cond(W)^2; the
    second pass, on the well-conditioned Q1, brings it to order eps.  Raises
    NotSPD when either Gram matrix is not positive definite."""
    Q1, R1 = cholqr(W, shift=shift)
    Q, R2 = cholqr(Q1)
    return Q, R2 @ R1


def assemble_pencil(S: list[np.ndarray], HS: list[np.ndarray]) -> tuple[np.ndarray, np.ndarray]:
    """G = S^T H S and O = S^T S from the lower blocks of eq. Glower.

    ``S`` and ``HS`` are lists of n x k blocks, e.g. [X, W, P] and [HX, HW, HP].
    Block (a, b) with a > b is S_a^T (H S_b); block (b, a) is its transpose.
    Diagonal blocks S_a^T H S_a are averaged with their transposes.
    """
    m = len(S)
    ks = [s.shape[1] for s in S]
    off = np.concatenate([[0], np.cumsum(ks)])
    N = int(off[-1])
    G = np.zeros((N, N))
    O = np.zeros((N, N))
    for a in range(m):
        for b in range(a + 1):
            ga = gram(S[a], HS[b])
            oa = gram(S[a], S[b])
            ra, rb = slice(off[a], off[a + 1]), slice(off[b], off[b + 1])
            if a == b:
                G[ra, ra] = 0.5 * (ga + ga.T)
                O[ra, ra] = 0.5 * (oa + oa.T)
            else:
                G[ra, rb] = ga
                G[rb, ra] = ga.T
                O[ra, rb] = oa
                O[rb, ra] = oa.T
    return G, O


def rayleigh_ritz(G: np.ndarray, O: np.ndarray, k: int) -> tuple[np.ndarray, np.ndarray]:
    """Solve G C = O C D (eq. rreig); return the k leftmost (theta, C), ascending.

    The pencil is first scaled to a unit diagonal of O (D = diag(O)^-1/2,
    G' = D G D, O' = D O D: the same eigenvalues, eigenvectors C = D C'), as
    if every basis column had unit norm; a Cholesky QR of an ill-conditioned W
    leaves columns whose norms are far from 1, and the unscaled reduction then
    loses the small directions of O.  Then O' = L L^T, A = L^{-1} G' L^{-T},
    A V = V D, C' = L^{-T} V.  Raises NotSPD if O is not positive definite or
    nearly singular: a squared pivot of L at or below RR_PIVOT_TOL.
    """
    dg = np.diag(O)
    if np.any(dg <= 0):
        raise NotSPD("zero column in the Rayleigh-Ritz basis")
    s = 1.0 / np.sqrt(dg)
    Gs = G * np.outer(s, s)
    Os = O * np.outer(s, s)
    R = cholesky_upper(Os)
    if np.min(np.diag(R)) ** 2 <= RR_PIVOT_TOL:
        raise NotSPD("nearly singular Rayleigh-Ritz basis")
    L = R.T
    Linv_G = sla.solve_triangular(L, Gs, lower=True)
    A = sla.solve_triangular(L, Linv_G.T, lower=True).T
    A = 0.5 * (A + A.T)
    d, V = np.linalg.eigh(A)
    C = sla.solve_triangular(L.T, V[:, :k], lower=False)
    return d[:k].copy(), C * s[:, None]
