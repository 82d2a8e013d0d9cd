"""Pins of the oracle's block-diagonal FOM preconditioner (Section 3.4):
FOM run for as many steps as the tile has rows is the exact tile solve; one
step has a closed form; the residual after m steps is orthogonal to the
Krylov space (the Galerkin condition that defines FOM), checked against a
basis built independently; the Arnoldi basis is orthonormal and projects A
onto H_m also on a tile dominated by a constant diagonal (where a single
Gram-Schmidt pass loses the basis); an eigenvector right-hand side ends the Arnoldi
process after one step with the exact solution; 1 x 1 tiles reproduce the
diagonal step; the dense diagonal tiles reassemble H."""
import numpy as np
import pytest

import synth
from oracle.precond import block_fom_precond, diag_precond, diagonal_tiles, fom


def sym(n, seed, shift=0.0):
    rng = np.random.default_rng(seed)
    M = rng.standard_normal((n, n))
    return (M + M.T) / 2 + shift * np.eye(n)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_full_steps_is_the_exact_solve(seed):
    A = sym(8, seed)
    lam = np.linalg.eigvalsh(A)
    sigma = 0.5 * (lam[3] + lam[4])          # indefinite shifted system, away from the spectrum
    b = np.random.default_rng(seed + 10).standard_normal(8)
    x, ok = fom(A - sigma * np.eye(8), b, 8)
    assert ok
    ref = np.linalg.solve(A - sigma * np.eye(8), b)
    assert np.abs(x - ref).max() <= 1e-9 * np.abs(ref).max()


def test_one_step_closed_form():
    A = sym(12, 3, shift=6.0)
    b = np.random.default_rng(4).standard_normal(12)
    x, ok = fom(A, b, 1)
    assert ok
    np.testing.assert_allclose(x, b * (b @ b) / (b @ A @ b), rtol=1e-13)


@pytest.mark.parametrize("m", [2, 3, 4])
def test_residual_orthogonal_to_krylov_space(m):
    A = sym(20, 5, shift=8.0)
    b = np.random.default_rng(6).standard_normal(20)
    x, ok = fom(A, b, m)
    assert ok
    # an independent orthonormal basis of span(b, Ab, ..., A^{m-1} b)
    K = np.stack([np.linalg.matrix_power(A, p) @ b for p in range(m)], axis=1)
    Q, _ = np.linalg.qr(K)
    r = b - A @ x
    assert np.abs(Q.T @ r).max() <= 1e-10 * np.linalg.norm(b)
    # and x lies in that space
    assert np.linalg.norm(x - Q @ (Q.T @ x)) <= 1e-10 * np.linalg.norm(x)


def test_arnoldi_basis_orthonormal_on_a_far_shifted_tile():
    """The Arnoldi process builds an orthonormal basis V_m with V_m^T A V_m =
    H_m.  On a diagonal tile of a block-sparse matrix shifted far below its
    spectrum (A = c I + E, |E| << c) every A v_j is nearly parallel to v_j; a
    single Gram-Schmidt pass loses the orthogonality of V_m there (V^T V off
    the identity by ~1) and this fails."""
    H = synth.tiled(64 * 40, tile=64, tile_draws=5, p=0.1, seed=2, f32=False)
    tiles = diagonal_tiles(H.n, H.row_ptr, H.col, H.val)
    A = tiles[5] + 1232.0 * np.eye(64)
    b = synth.gaussian_block(H.n, 8, seed=5)[5 * 64:6 * 64, 0]
    x, ok, V, Hs = fom(A, b, 8, basis=True)
    assert ok and V.shape == (64, 8)
    assert np.abs(V.T @ V - np.eye(8)).max() <= 1e-13
    assert np.abs(V.T @ A @ V - Hs).max() <= 1e-12 * np.abs(A).max()
    # and the Galerkin condition on the iterate
    assert np.abs(V.T @ (b - A @ x)).max() <= 1e-12 * np.linalg.norm(b)


def test_eigenvector_right_hand_side_is_solved_in_one_step():
    A = sym(16, 7, shift=3.0)
    lam, V = np.linalg.eigh(A)
    b = 2.5 * V[:, 5]
    x, ok = fom(A, b, 4)
    assert ok
    np.testing.assert_allclose(x, b / lam[5], rtol=1e-10, atol=1e-12)


def test_singular_hessenberg_reports_no_iterate():
    A = np.diag([1.0, -1.0])
    b = np.array([1.0, 1.0])                 # b^T A b = 0: the 1 x 1 Hessenberg is zero
    x, ok = fom(A, b, 1)
    assert not ok


def test_one_by_one_tiles_are_the_diagonal_step():
    rng = np.random.default_rng(8)
    n, k = 30, 4
    d = rng.uniform(5.0, 9.0, n)
    A = synth.diagonal(d)
    tiles = diagonal_tiles(n, A.row_ptr, A.col, A.val, tile=1)
    R = rng.standard_normal((n, k))
    theta = np.array([1.0, 1.5, 2.0, 2.5])
    for off in (0.0, 2.0):
        W = block_fom_precond(tiles, R, theta, 3, eps=1e-6, offset=off)
        np.testing.assert_allclose(W, diag_precond(R, d, theta, 1e-6, off), rtol=1e-14)
    # a zero divisor has no FOM iterate: the guarded diagonal step is used
    theta0 = np.array([d[4], 1.0, 1.0, 1.0])
    W = block_fom_precond(tiles, R, theta0, 3, eps=1e-6)
    np.testing.assert_array_equal(W[4, 0], R[4, 0] / 1e-6)


def test_tiles_reassemble_h_and_blocks_solve_exactly():
    """Diagonal tiles of a random symmetric matrix (n = 10, tiles of 4: the last
    one ragged) equal the dense blocks of H; with m = 4 FOM steps every block
    is solved exactly: W_t = (H_tt - sigma_j I)^{-1} R_t."""
    A = synth.random_sym(10, 3, seed=2)
    Hd = np.zeros((10, 10))
    for i in range(10):
        for e in range(A.row_ptr[i], A.row_ptr[i + 1]):
            Hd[i, A.col[e]] = Hd[A.col[e], i] = A.val[e]
    tiles = diagonal_tiles(10, A.row_ptr, A.col, A.val, tile=4)
    assert tiles.shape == (3, 4, 4)
    for t in range(3):
        lo, hi = 4 * t, min(10, 4 * t + 4)
        np.testing.assert_array_equal(tiles[t][:hi - lo, :hi - lo], Hd[lo:hi, lo:hi])
    np.testing.assert_array_equal(tiles[2][2:, 2:], np.eye(2))
    rng = np.random.default_rng(3)
    R = rng.standard_normal((10, 2))
    theta = np.array([-7.3, -5.1])
    W = block_fom_precond(tiles, R, theta, 4, eps=1e-9)
    for t in range(3):
        lo, hi = 4 * t, min(10, 4 * t + 4)
        for j in range(2):
            ref = np.linalg.solve(Hd[lo:hi, lo:hi] - theta[j] * np.eye(hi - lo), R[lo:hi, j])
            np.testing.assert_allclose(W[lo:hi, j], ref, rtol=1e-9, atol=1e-12)
