"""Pins for the FP64 oracle SpMM Y = (U + U^T - diag U) X (Algorithm 2 and
Section 3.2: the stored part and its transpose).  Each pin checks the oracle
against something other than itself: SciPy's sparse product (a library
routine), a dense brute-force product on tiny integer matrices, algebraic
identities, and special cases."""
import numpy as np
import pytest
import scipy.sparse as sp

import oracle
import synth


def scipy_full(A):
    U = sp.csr_matrix((np.asarray(A.val, dtype=np.float64), A.col, A.row_ptr), shape=(A.n, A.n))
    return (U + U.T - sp.diags(U.diagonal())).tocsr()


@pytest.mark.parametrize("maker", [
    lambda: synth.random_sym(3000, 20, seed=3),
    lambda: synth.random_sym(3000, 20, seed=4, f32=True),
    lambda: synth.tiled(64 * 40, tile=64, tile_draws=5, p=0.1, seed=2),
    lambda: synth.zipf(4000, lmin=4, lmax=400, seed=5),
])
@pytest.mark.parametrize("k", [1, 8, 16])
def test_matches_scipy(maker, k):
    A = maker()
    H = oracle.SymMatrix.from_csr(A)
    X = synth.gaussian_block(A.n, k, seed=11)
    Y = H @ X
    Yref = scipy_full(A) @ X
    np.testing.assert_allclose(Y, Yref, rtol=1e-12, atol=1e-12 * np.abs(Yref).max())


def test_tiny_integer_bruteforce():
    rng = np.random.default_rng(0)
    n, k = 9, 3
    Hd = np.triu(rng.integers(-4, 5, size=(n, n)).astype(float))
    Hd[rng.random((n, n)) < 0.5] = 0.0
    Hd = Hd + np.triu(Hd, 1).T
    np.fill_diagonal(Hd, rng.integers(1, 9, size=n))
    A = synth.from_dense_upper(Hd)
    X = rng.integers(-5, 6, size=(n, k)).astype(float)
    Y = oracle.SymMatrix.from_csr(A) @ X
    # integer data: any summation order is exact
    assert np.array_equal(Y, Hd @ X)


def test_diagonal_only():
    d = np.linspace(-3, 7, 50)
    A = synth.diagonal(d)
    X = synth.gaussian_block(50, 4, seed=2)
    assert np.array_equal(oracle.SymMatrix.from_csr(A) @ X, d[:, None] * X)


def test_symmetry_identity():
    A = synth.random_sym(2000, 15, seed=7)
    H = oracle.SymMatrix.from_csr(A)
    X = synth.gaussian_block(A.n, 5, seed=1)
    Y = synth.gaussian_block(A.n, 6, seed=2)
    lhs = X.T @ (H @ Y)
    rhs = (H @ X).T @ Y
    np.testing.assert_allclose(lhs, rhs, rtol=1e-11, atol=1e-9)


def test_permutation_invariance():
    A = synth.random_sym(500, 12, seed=9)
    Hd = scipy_full(A).toarray()
    perm = np.random.default_rng(1).permutation(A.n)
    Hp = Hd[np.ix_(perm, perm)]
    Ap = synth.from_dense_upper(Hp)
    X = synth.gaussian_block(A.n, 3, seed=4)
    Y = oracle.SymMatrix.from_csr(A) @ X
    Yp = oracle.SymMatrix.from_csr(Ap) @ X[perm]
    np.testing.assert_allclose(Yp, Y[perm], rtol=1e-12, atol=1e-12)


def test_rows_and_abs():
    A = synth.random_sym(1500, 10, seed=12)
    H = oracle.SymMatrix.from_csr(A)
    X = synth.gaussian_block(A.n, 8, seed=3)
    rows = np.array([0, 1, 17, 700, 1499])
    Yr, Ya = H.rows(X, rows)
    np.testing.assert_allclose(Yr, (H @ X)[rows], rtol=1e-13, atol=1e-13)
    Habs = abs(scipy_full(A))
    np.testing.assert_allclose(Ya, (Habs @ np.abs(X))[rows], rtol=1e-13)
    np.testing.assert_allclose(H.abs_matmul(X), Habs @ np.abs(X), rtol=1e-13)


def test_gershgorin_and_row_norms():
    A = synth.random_sym(800, 9, seed=13)
    Hd = scipy_full(A).toarray()
    H = oracle.SymMatrix.from_csr(A)
    assert H.gershgorin() == pytest.approx(np.abs(Hd).sum(axis=1).max(), rel=1e-13)
    off = np.abs(Hd).sum(axis=1) - np.abs(np.diag(Hd))
    np.testing.assert_allclose(H.row_offdiag_abs(), off, rtol=1e-13, atol=1e-13)
    np.testing.assert_array_equal(H.row_offdiag_count(), (Hd != 0).sum(axis=1) - (np.diag(Hd) != 0))


def test_generator_shapes():
    """The generated matrices are upper-triangular CSR, sorted, diagonal first."""
    for A in (synth.random_sym(1000, 50, seed=0), synth.tiled(64 * 30, tile_draws=4, p=0.1, seed=1),
              synth.zipf(3000, lmin=4, lmax=300, seed=2)):
        rl = np.diff(A.row_ptr)
        rows = np.repeat(np.arange(A.n), rl)
        assert (A.col >= rows).all()
        assert (A.col[A.row_ptr[:-1]] == np.arange(A.n)).all()
        for i in range(0, A.n, 37):
            seg = A.col[A.row_ptr[i]:A.row_ptr[i + 1]]
            assert (np.diff(seg) > 0).all()
        assert np.all(np.diff(A.diag) >= 0)


def test_thread_count_does_not_change_result():
    """Both passes pull into their own output rows, so the product is the same
    bits on one thread and on all of them."""
    A = synth.random_sym(20000, 30, seed=11)
    H = oracle.SymMatrix.from_csr(A)
    X = np.random.default_rng(4).standard_normal((A.n, 5))
    full = oracle.threads()
    Y = H @ X
    oracle.set_threads(1)
    try:
        assert oracle.threads() == 1
        Y1 = H @ X
    finally:
        oracle.set_threads(full)
    assert oracle.threads() == full
    assert np.array_equal(Y, Y1)
