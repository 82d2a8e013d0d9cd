"""Pins for the oracle's FP64 dense steps: Cholesky QR (Section 3.5), the
pencil assembled from lower blocks (eq. Glower) and Rayleigh-Ritz (eq. rreig),
against LAPACK's generalized solver (scipy.linalg.eigh(G, O) calls dsygv, the
routine the paper uses), a closed-form 2x2 pencil, and the defining identities."""
import numpy as np
import pytest
import scipy.linalg as sla

import oracle
import synth
from oracle.dense import NotSPD, assemble_pencil, cholqr, rayleigh_ritz
from oracle.precond import diag_precond, guard


def random_pencil(N, seed):
    rng = np.random.default_rng(seed)
    G = rng.standard_normal((N, N))
    G = G + G.T
    B = rng.standard_normal((N, N))
    O = B @ B.T + N * np.eye(N)
    return G, O


@pytest.mark.parametrize("N,k", [(8, 8), (24, 8), (48, 16), (16, 5)])
def test_rr_matches_dsygv(N, k):
    G, O = random_pencil(N, N + k)
    theta, C = rayleigh_ritz(G, O, k)
    ref = sla.eigh(G, O, eigvals_only=True)[:k]
    np.testing.assert_allclose(theta, ref, rtol=1e-11, atol=1e-11)
    np.testing.assert_allclose(C.T @ O @ C, np.eye(k), atol=1e-10)
    np.testing.assert_allclose(C.T @ G @ C, np.diag(theta), atol=1e-9)
    assert np.all(np.diff(theta) >= 0)


def test_rr_closed_form_2x2():
    # G = [[a, b], [b, c]], O = I: eigenvalues (a+c)/2 -+ sqrt(((a-c)/2)^2 + b^2)
    a, b, c = 3.0, -1.25, 0.5
    theta, _ = rayleigh_ritz(np.array([[a, b], [b, c]]), np.eye(2), 2)
    r = np.hypot((a - c) / 2, b)
    np.testing.assert_allclose(theta, [(a + c) / 2 - r, (a + c) / 2 + r], rtol=1e-14)
    # scaled metric O = diag(s): eigenvalues of diag(s)^-1/2 G diag(s)^-1/2
    s = np.array([4.0, 0.25])
    G = np.array([[a, b], [b, c]])
    theta2, _ = rayleigh_ritz(G, np.diag(s), 2)
    Gs = G / np.sqrt(np.outer(s, s))
    r2 = np.hypot((Gs[0, 0] - Gs[1, 1]) / 2, Gs[0, 1])
    np.testing.assert_allclose(theta2, [(Gs[0, 0] + Gs[1, 1]) / 2 - r2, (Gs[0, 0] + Gs[1, 1]) / 2 + r2],
                               rtol=1e-13)


def test_rr_not_spd_raises():
    G = np.eye(3)
    O = np.diag([1.0, 0.0, 1.0])
    with pytest.raises(NotSPD):
        rayleigh_ritz(G, O, 2)


def test_cholqr():
    W = synth.gaussian_block(500, 8, seed=3) * np.array([1, 2, 3, 1e-3, 5, 6, 7, 8.0])
    Q, R = cholqr(W)
    np.testing.assert_allclose(Q.T @ Q, np.eye(8), atol=1e-12)
    np.testing.assert_allclose(Q @ R, W, atol=1e-12)
    assert np.allclose(R, np.triu(R))
    with pytest.raises(NotSPD):
        cholqr(np.hstack([W[:, :3], W[:, :1]]))


def test_pencil_from_lower_blocks():
    A = synth.random_sym(600, 10, seed=21)
    H = oracle.SymMatrix.from_csr(A)
    blocks = [synth.gaussian_block(A.n, 4, seed=s) for s in (1, 2, 3)]
    HB = [H @ b for b in blocks]
    G, O = assemble_pencil(blocks, HB)
    S = np.hstack(blocks)
    HS = H @ S
    np.testing.assert_allclose(G, S.T @ HS, rtol=1e-11, atol=1e-9)
    np.testing.assert_allclose(O, S.T @ S, rtol=1e-12, atol=1e-9)
    assert np.array_equal(G, G.T) and np.array_equal(O, O.T)


def test_diag_precond_closed_form():
    d = np.array([0.0, 1.0, 2.0, 10.0])
    theta = np.array([-1.0, 1.0])
    R = np.ones((4, 2))
    eps = 0.5
    W = diag_precond(R, d, theta, eps)
    expect = np.array([[1 / 1.0, 1 / -1.0 if False else 1 / 0.5],
                       [1 / 2.0, 1 / 0.5],
                       [1 / 3.0, 1 / 1.0],
                       [1 / 11.0, 1 / 9.0]])
    # d - theta for column 1 = [-1, 0, 1, 9]: -1 kept (|-1| >= eps), 0 -> +eps
    expect[0, 1] = 1 / -1.0
    np.testing.assert_allclose(W, expect, rtol=1e-15)
    np.testing.assert_array_equal(guard(np.array([0.0, -0.1, 0.1, -2.0]), 0.5), [0.5, -0.5, 0.5, -2.0])


def test_shifted_cholqr():
    W = synth.gaussian_block(400, 6, seed=9)
    W = np.hstack([W, W[:, :1] * (1 + 1e-15)])   # numerically dependent column
    with pytest.raises(NotSPD):
        cholqr(W)
    Q, R = cholqr(W, shift=1e-12)
    np.testing.assert_allclose(Q @ R, W, atol=1e-10)
    # the well-conditioned part stays orthonormal
    np.testing.assert_allclose(Q[:, :6].T @ Q[:, :6], np.eye(6), atol=1e-8)
    # the shift is a no-op for a well-conditioned block (up to the shift itself)
    W2 = synth.gaussian_block(400, 5, seed=10)
    Q1, _ = cholqr(W2)
    Q2, _ = cholqr(W2, shift=1e-12)
    np.testing.assert_allclose(Q1, Q2, atol=1e-10)


def _conditioned(n, k, cond, seed):
    """n x k matrix with singular values spaced geometrically from 1 to 1/cond."""
    rng = np.random.default_rng(seed)
    U, _ = np.linalg.qr(rng.standard_normal((n, k)))
    V, _ = np.linalg.qr(rng.standard_normal((k, k)))
    return (U * np.geomspace(1.0, 1.0 / cond, k)) @ V.T


def test_cholqr2_orthogonality_and_factor():
    """CholeskyQR2 (Fukaya et al. 2014): on W with cond(W) = 1e6 one Cholesky
    QR leaves an orthogonality error of order eps cond^2 (here above 1e-8);
    the second pass brings it to order eps.  W = Q R with R upper triangular."""
    from oracle.dense import cholqr2
    W = _conditioned(2000, 8, 1e6, seed=3)
    Q1, _ = cholqr(W)
    e1 = np.abs(Q1.T @ Q1 - np.eye(8)).max()
    Q, R = cholqr2(W)
    e2 = np.abs(Q.T @ Q - np.eye(8)).max()
    assert e1 > 1e-8 and e2 < 1e-14, (e1, e2)
    assert np.allclose(np.tril(R, -1), 0.0)
    assert np.abs(Q @ R - W).max() <= 1e-14 * np.abs(W).max()


def test_cholqr2_shifted_first_pass():
    """At cond(W) = 1e9 (cond^2 beyond 1/eps) the plain Gram matrix is not
    positive definite to the Cholesky factorisation; a shifted first pass and
    a plain second one give W = Q R with Q orthonormal to 1e-11 (the shifted
    pass leaves Q1 with a condition number of about shift^-1/2), and one more
    plain pass (shifted CholeskyQR3, Fukaya et al. 2020) to eps."""
    from oracle.dense import cholqr2
    W = _conditioned(2000, 8, 1e9, seed=4)
    with pytest.raises(NotSPD):
        cholqr(W)
    Q, R = cholqr2(W, shift=1e-12)
    assert np.abs(Q.T @ Q - np.eye(8)).max() < 1e-11
    assert np.abs(Q @ R - W).max() <= 1e-14 * np.abs(W).max()
    Q3, _ = cholqr(Q)
    assert np.abs(Q3.T @ Q3 - np.eye(8)).max() < 1e-14


@pytest.mark.parametrize("orthonormal_x", [True, False])
def test_projected_gram_from_one_gram_of_x_and_w(orthonormal_x):
    """The identity the GPU's one-pass orthogonalisation uses (Section 3.5's
    projection W - X (X^T W) followed by Cholesky QR): with C = X^T W,
    (W - X C)^T (W - X C) = W^T W - C^T C - C^T C + C^T (X^T X) C for any X,
    so the Gram of [X W] alone gives the projected block's Gram, and
    W R^{-1} - X (C R^{-1}) is the oracle's Q of the projected block."""
    rng = np.random.default_rng(11)
    n, k = 300, 6
    X = rng.standard_normal((n, k))
    if orthonormal_x:
        X, _ = np.linalg.qr(X)
    W = rng.standard_normal((n, k)) + X @ (3.0 * rng.standard_normal((k, k)))
    C = X.T @ W
    Wp = W - X @ C
    B_direct = Wp.T @ Wp
    B_formula = W.T @ W - C.T @ C - C.T @ C + C.T @ (X.T @ X) @ C
    scale = np.abs(W.T @ W).max() + np.abs(C.T @ (X.T @ X) @ C).max()
    assert np.abs(B_direct - B_formula).max() <= 1e-12 * scale
    Q, R = cholqr(Wp)
    Rf = np.linalg.cholesky(0.5 * (B_formula + B_formula.T)).T
    Q_formula = W @ np.linalg.inv(Rf) - X @ (C @ np.linalg.inv(Rf))
    assert np.abs(Q - Q_formula).max() <= 1e-9
    assert np.abs(Q.T @ Q - np.eye(k)).max() <= 1e-12
