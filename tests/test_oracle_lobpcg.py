"""Pins for the oracle's LOBPCG (Algorithm 1 with the recurrences eqs. upd1-upd2
and Cholesky QR of Section 3.5): dense LAPACK eigh at n <= 2000, ARPACK at
n = 20,000, closed-form spectra, and invariants (orthonormal X, Ritz values
non-increasing, the residual bound |theta - lambda| <= ||r|| / ||x||)."""
import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla

import oracle
import synth
from oracle.lobpcg import ENOCONV, OK, lobpcg
from synth import workloads as W


def dense(A):
    U = sp.csr_matrix((np.asarray(A.val, dtype=np.float64), A.col, A.row_ptr), shape=(A.n, A.n))
    return (U + U.T - sp.diags(U.diagonal())).toarray()


def solve(A, k=8, nev=5, **kw):
    H = oracle.SymMatrix.from_csr(A)
    X0 = W.initial_block(A.n, k, seed=1)
    return H, lobpcg(H, X0, nev, d=A.diag, **kw)


def test_random_sym_1k_vs_dense_eigh():
    A = W.make_matrix("random_sym_1k")
    H, r = solve(A)
    assert r.status == OK
    lam = np.linalg.eigvalsh(dense(A))[:5]
    np.testing.assert_allclose(r.theta, lam, rtol=1e-9)
    # invariants along the way
    th = np.array(r.theta_hist)
    gamma = H.gershgorin()
    assert np.all(np.diff(th, axis=0) <= 1e-12 * gamma)          # Ritz values never increase
    np.testing.assert_allclose(r.X_all.T @ r.X_all, np.eye(8), atol=1e-10)
    # residual certificate for each returned pair
    res = H @ r.X - r.X * r.theta
    bound = np.linalg.norm(res, axis=0) / np.linalg.norm(r.X, axis=0)
    assert np.all(np.abs(r.theta - lam) <= bound * (1 + 1e-6) + 1e-12)


def test_subspace_matches_eigh():
    A = synth.random_sym(800, 30, seed=5)
    Hd = dense(A)
    H, r = solve(A, tol=1e-9)
    assert r.status == OK
    lam, V = np.linalg.eigh(Hd)
    # principal angles between span(X) and the exact invariant subspace
    s = np.linalg.svd(V[:, :5].T @ r.X, compute_uv=False)
    assert s.min() > 1 - 1e-9


@pytest.mark.slow
def test_random_sym_20k_vs_arpack():
    A = W.make_matrix("random_sym_20k")
    H, r = solve(A)
    assert r.status == OK
    U = sp.csr_matrix((A.val, A.col, A.row_ptr), shape=(A.n, A.n))
    Hs = U + U.T - sp.diags(U.diagonal())
    lam = np.sort(spla.eigsh(Hs, k=6, which="SA", tol=1e-13)[0])[:5]
    np.testing.assert_allclose(r.theta, lam, rtol=1e-7)


def test_diagonal_matrix_one_step():
    d = np.sort(np.random.default_rng(0).uniform(0, 10, 300))
    A = synth.diagonal(d)
    H = oracle.SymMatrix.from_csr(A)
    # start from a block that is a permutation of unit vectors around the lowest ones
    X0 = np.zeros((300, 8))
    X0[np.arange(8), np.arange(8)[::-1]] = 1.0
    r = lobpcg(H, X0, 5, d=A.diag)
    assert r.status == OK and r.iters == 0
    np.testing.assert_allclose(r.theta, d[:5], rtol=1e-15)


def test_laplacian_closed_form():
    n = 120
    A = synth.laplacian_1d(n)
    H = oracle.SymMatrix.from_csr(A)
    r = lobpcg(H, W.initial_block(n, 8, seed=1), 5, tol=1e-10, precond=None, maxiter=3000)
    assert r.status == OK
    j = np.arange(1, 6)
    np.testing.assert_allclose(r.theta, 2 - 2 * np.cos(j * np.pi / (n + 1)), rtol=1e-8)


def test_blocks_2x2_closed_form():
    rng = np.random.default_rng(3)
    m = 100
    a, c = rng.uniform(0, 10, m), rng.uniform(0, 10, m)
    b = rng.uniform(-2, 2, m)
    A = synth.blocks_2x2(a, b, c)
    H = oracle.SymMatrix.from_csr(A)
    r = lobpcg(H, W.initial_block(2 * m, 8, seed=1), 5, tol=1e-10, d=A.diag)
    assert r.status == OK
    lo = (a + c) / 2 - np.hypot((a - c) / 2, b)
    hi = (a + c) / 2 + np.hypot((a - c) / 2, b)
    lam = np.sort(np.concatenate([lo, hi]))[:5]
    np.testing.assert_allclose(r.theta, lam, rtol=1e-9, atol=1e-12)


def test_maxiter_exhaustion():
    A = W.make_matrix("random_sym_1k")
    H, r = solve(A, maxiter=3)
    assert r.status == ENOCONV and r.iters == 3
    assert len(r.theta_hist) == 3


def test_recurrence_tracks_explicit_product():
    """H X carried by eqs. upd1-upd2 stays close to the explicit product."""
    A = synth.random_sym(1000, 30, seed=8)
    H = oracle.SymMatrix.from_csr(A)
    seen = {}

    def cb(it, X, R, theta, Wb):
        seen["X"], seen["R"], seen["theta"] = X.copy(), R.copy(), theta.copy()
    r = lobpcg(H, W.initial_block(A.n, 8, seed=1), 5, d=A.diag, maxiter=40, callback=cb)
    X, R, theta = seen["X"], seen["R"], seen["theta"]
    Rexp = H @ X - X * theta
    assert np.abs(R - Rexp).max() < 1e-10 * H.gershgorin()


def test_precond_offset_by_hand():
    """sigma_j = theta_j - c (max theta - min theta), W_ij = R_ij / s(d_i - sigma_j)."""
    from oracle.precond import diag_precond
    R = np.array([[1.0, 2.0], [3.0, -4.0]])
    d = np.array([1.0, 4.0])
    theta = np.array([1.5, 0.5])                 # spread 1.0, unsorted on purpose
    # c = 0: divisors d - theta = [[-0.5, 0.5], [2.5, 3.5]]
    np.testing.assert_array_equal(diag_precond(R, d, theta, 1e-3), R / np.array([[-0.5, 0.5], [2.5, 3.5]]))
    # c = 2: sigma = [-0.5, -1.5], divisors [[1.5, 2.5], [4.5, 5.5]]
    np.testing.assert_array_equal(diag_precond(R, d, theta, 1e-3, offset=2.0),
                                  R / np.array([[1.5, 2.5], [4.5, 5.5]]))
    # the guard still applies to the shifted divisor: d_0 - sigma_0 = 0 -> +eps
    W = diag_precond(R, d, np.array([1.0, 1.0]), 0.25, offset=3.0)   # spread 0: sigma = theta
    np.testing.assert_array_equal(W[0], R[0] / 0.25)


@pytest.mark.parametrize("offset", [1.0, 2.0])
def test_precond_offset_solve_vs_dense_eigh(offset):
    """The shift moved below the Ritz values changes the iterates, not the
    answer: the same eigenvalues as dense LAPACK, fewer iterations than the
    shift at the Ritz value on this matrix."""
    A = W.make_matrix("random_sym_1k")
    lam = np.linalg.eigvalsh(dense(A))[:5]
    H, r0 = solve(A)
    H, r = solve(A, precond_offset=offset)
    assert r.status == OK
    np.testing.assert_allclose(r.theta, lam, rtol=1e-9)
    np.testing.assert_allclose(r.X_all.T @ r.X_all, np.eye(8), atol=1e-10)
    assert r.iters < r0.iters, (r.iters, r0.iters)


def test_near_diagonal_shift_at_theta_keeps_ritz_values_in_the_spectrum():
    """Nearly diagonal H with the diagonal step's shift at theta_j: the basis
    [X, W, P] drifts toward dependence and the Rayleigh-Ritz Gram O becomes
    nearly singular (scaled pivots ~1e-14 here).  Accepting such an O gives
    Ritz values below the lowest eigenvalue (Courant-Fischer forbids them for
    an exact projection); the oracle drops P instead and converges to the
    dense spectrum."""
    A = synth.near_diagonal(2000)
    H = oracle.SymMatrix.from_csr(A)
    lam = np.linalg.eigvalsh(H @ np.eye(A.n))
    r = lobpcg(H, W.initial_block(A.n, 8, seed=1), 5, d=A.diag, maxiter=2000)
    assert r.status == OK
    assert r.p_dropped > 0
    assert np.min(np.array(r.theta_hist)) >= lam[0] - 1e-12 * H.gershgorin()
    np.testing.assert_allclose(r.theta, lam[:5], rtol=1e-8)


def test_rayleigh_ritz_rejects_a_nearly_singular_basis():
    """Two basis columns at an angle of 1e-6 (scaled Gram pivot ~1e-12): the
    Rayleigh-Ritz step reports a non-SPD O; at an angle of 1e-3 (pivot 1e-6) it
    proceeds and its Ritz values lie inside the spectrum of H."""
    from oracle.dense import NotSPD, assemble_pencil, rayleigh_ritz
    rng = np.random.default_rng(4)
    n = 50
    M = rng.standard_normal((n, n))
    Hd = M + M.T
    lam = np.linalg.eigvalsh(Hd)
    for angle, ok in ((1e-6, False), (1e-3, True)):
        S = rng.standard_normal((n, 3))
        S[:, 2] = S[:, 1] + angle * np.linalg.norm(S[:, 1]) * rng.standard_normal(n) / np.sqrt(n)
        G, O = assemble_pencil([S], [Hd @ S])
        if ok:
            th, C = rayleigh_ritz(G, O, 3)
            assert np.all(th >= lam[0] - 1e-9) and np.all(th <= lam[-1] + 1e-9)
        else:
            with pytest.raises(NotSPD):
                rayleigh_ritz(G, O, 3)


def test_cholqr2_solve_vs_dense_eigh():
    """LOBPCG with CholeskyQR2 for W: the same eigenpairs as dense eigh, Ritz
    values never increasing, and an iteration count close to the one-pass
    solve's (the second pass changes W only at the rounding level here)."""
    A = W.make_matrix("random_sym_1k")
    H, r1 = solve(A)
    _, r2 = solve(A, cholqr_passes=2)
    assert r2.status == OK
    lam = np.linalg.eigvalsh(dense(A))[:5]
    np.testing.assert_allclose(r2.theta, lam, rtol=1e-9)
    th = np.array(r2.theta_hist)
    assert np.all(np.diff(th, axis=0) <= 1e-12 * H.gershgorin())
    assert abs(r2.iters - r1.iters) <= 0.1 * r1.iters, (r1.iters, r2.iters)


def test_soft_lock_solve():
    """Soft locking: a column whose relative residual was <= tol at the last
    check leaves W and P.  The solve still finds the dense eigenpairs, the
    Ritz values never increase (X stays in every Rayleigh-Ritz basis), and the
    W of each iteration has exactly the columns not converged at the previous
    check (seen by the callback)."""
    A = W.make_matrix("random_sym_1k")
    widths = []
    H, r = solve(A, soft_lock=True, callback=lambda it, X, R, th, Wb: widths.append(Wb.shape[1]))
    assert r.status == OK
    lam = np.linalg.eigvalsh(dense(A))[:5]
    np.testing.assert_allclose(r.theta, lam, rtol=1e-9)
    th = np.array(r.theta_hist)
    assert np.all(np.diff(th, axis=0) <= 1e-12 * H.gershgorin())
    assert widths == r.active_hist
    # active widths follow the previous iteration's residuals
    rel = np.array(r.rel_hist)
    for i in range(1, len(widths)):
        assert widths[i] == int(np.sum(rel[i - 1] > 1e-6))
    assert min(widths) < 8                    # some column was locked before the end
    np.testing.assert_allclose(r.X_all.T @ r.X_all, np.eye(8), atol=1e-10)
