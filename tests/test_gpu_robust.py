"""CholeskyQR2 and soft locking on the GPU (Section 3.5; the FP32 drift of
eqs. upd1-upd2) against the FP64 oracle: lobpcg_cholqr on blocks of known
condition number against oracle.dense.cholqr / cholqr2, and solves with
lobpcg_set_cholqr_passes(2) and lobpcg_set_soft_lock(1) against the oracle's
LOBPCG with the same options (eigenvalues, iteration counts, and the Ritz
value history on a matrix with separated wanted eigenvalues)."""
import numpy as np
import pytest

import oracle
import synth
from gpu_util import to_dev, torch_cuda, upload
from oracle.dense import NotSPD, cholqr, cholqr2
from oracle.lobpcg import lobpcg as oracle_lobpcg
from synth import workloads as W

pytestmark = pytest.mark.gpu


def conditioned(n, k, cond, seed):
    rng = np.random.default_rng(seed)
    U, _ = np.linalg.qr(rng.standard_normal((n, k)))
    V, _ = np.linalg.qr(rng.standard_normal((k, k)))
    return (U * np.geomspace(1.0, 1.0 / cond, k)) @ V.T


def orth_error(Q):
    return float(np.abs(Q.T @ Q - np.eye(Q.shape[1])).max())


def test_cholqr_one_and_two_passes():
    """cond(W) = 1e6, FP64: one pass leaves an orthogonality error of order
    eps cond^2 like the oracle's; two passes reach eps, and Q is the oracle's
    CholeskyQR2 factor (the Q of a QR factorisation with positive R diagonal
    is unique; both agree to about eps cond)."""
    torch_cuda()
    A = W.make_matrix("random_sym_1k")
    ctx = upload(A, False)
    Wm = conditioned(A.n, 8, 1e6, seed=3)
    Q1 = to_dev(Wm, np.float64)
    assert ctx.cholqr(Q1, passes=1) == 0
    e1, e1_ref = orth_error(Q1.cpu().numpy()), orth_error(cholqr(Wm)[0])
    Q2 = to_dev(Wm, np.float64)
    assert ctx.cholqr(Q2, passes=2) == 0
    Q2n = Q2.cpu().numpy()
    Qref, _ = cholqr2(Wm)
    print(f"orthogonality: one pass {e1:.2e} (oracle {e1_ref:.2e}), two passes {orth_error(Q2n):.2e}")
    assert 1e-8 < e1 < 1e-2 and 0.01 < e1 / e1_ref < 100
    assert orth_error(Q2n) < 1e-14
    assert np.abs(Q2n - Qref).max() < 1e-8


def test_cholqr_shifted_pass_and_fp32():
    """cond(W) = 1e10 in FP64: the plain Gram fails, the first pass is shifted
    (counted) and the second plain one leaves Q orthonormal to about 1e-10, as
    in the oracle (1.0e-10).  FP32 context, cond 1e3: two passes orthonormal to
    FP32 rounding."""
    import paper_2109_00485_amd as L
    torch_cuda()
    A = W.make_matrix("random_sym_1k")
    ctx = upload(A, False)
    Wm = conditioned(A.n, 8, 1e10, seed=4)
    with pytest.raises(NotSPD):
        cholqr(Wm)
    Q = to_dev(Wm, np.float64)
    assert ctx.cholqr(Q, passes=2) == 1
    e = orth_error(Q.cpu().numpy())
    e_ref = orth_error(cholqr2(Wm, shift=1e-12)[0])
    print(f"shifted first pass: orthogonality {e:.2e} (oracle {e_ref:.2e})")
    assert e < 1e-9
    ctx32 = upload(A, True)
    Wf = conditioned(A.n, 8, 1e3, seed=5).astype(np.float32)
    Qf = to_dev(Wf, np.float32)
    ctx32.cholqr(Qf, passes=2)
    assert orth_error(Qf.cpu().numpy().astype(np.float64)) < 2e-6
    with pytest.raises(L.LobpcgError):
        ctx.cholqr(Q, passes=3)


def dense_lowest(A, nev=5):
    H = oracle.SymMatrix.from_csr(A)
    return np.linalg.eigvalsh(H @ np.eye(A.n))[:nev], H


@pytest.mark.parametrize("f32", [False, True])
def test_cholqr2_solve(f32):
    A = W.make_matrix("random_sym_1k")
    lam, H = dense_lowest(A)
    ref = oracle_lobpcg(H, W.initial_block(A.n, 8, seed=1), 5, d=A.diag, cholqr_passes=2)
    ctx = upload(A, f32)
    ctx.set_cholqr_passes(2)
    dt = np.float32 if f32 else np.float64
    X = to_dev(W.initial_block(A.n, 8, seed=1), dt)
    r = ctx.solve(X, 5, tol=3e-6 if f32 else 1e-6, maxiter=3000)
    print(f"f32={f32}: {r.iters} iterations (oracle {ref.iters})")
    assert r.status == 0
    tau = 1e-3 * H.gershgorin()
    assert np.all(np.abs(r.evals[:5] - lam) <= 1e-6 * np.maximum(np.abs(lam), tau)), (r.evals[:5], lam)
    if not f32:
        assert abs(r.iters - ref.iters) <= 0.15 * ref.iters


@pytest.mark.parametrize("f32", [False, True])
def test_soft_lock_solve(f32):
    """Soft locking: the same eigenpairs as dense eigh and as the oracle's
    soft-locked LOBPCG, with columns locked along the way (locked_max > 0)."""
    A = W.make_matrix("random_sym_1k")
    lam, H = dense_lowest(A)
    ref = oracle_lobpcg(H, W.initial_block(A.n, 8, seed=1), 5, d=A.diag, soft_lock=True)
    ctx = upload(A, f32)
    ctx.set_soft_lock(True)
    dt = np.float32 if f32 else np.float64
    X = to_dev(W.initial_block(A.n, 8, seed=1), dt)
    r = ctx.solve(X, 5, tol=3e-6 if f32 else 1e-6, maxiter=3000)
    print(f"f32={f32}: {r.iters} iterations (oracle {ref.iters}), at most {r.locked_max} columns locked")
    assert r.status == 0 and r.locked_max > 0
    tau = 1e-3 * H.gershgorin()
    assert np.all(np.abs(r.evals[:5] - lam) <= 1e-6 * np.maximum(np.abs(lam), tau)), (r.evals[:5], lam)
    Xg = X.cpu().numpy().astype(np.float64)
    assert np.abs(Xg.T @ Xg - np.eye(8)).max() < (2e-5 if f32 else 1e-10)


def test_soft_lock_history_matches_oracle():
    """On the matrix with separated wanted eigenvalues (FP64, shift 4 spreads
    below theta_j), every iteration's Ritz values of the soft-locked GPU solve
    against the soft-locked oracle's, bar 1e-9 relative as for the plain
    solve: the locking decisions (rel_j <= tol) fall the same way on both."""
    A = synth.near_diagonal(2000)
    H = oracle.SymMatrix.from_csr(A)
    ref = oracle_lobpcg(H, W.initial_block(A.n, 8, seed=1), 5, d=A.diag, precond_offset=4.0, soft_lock=True)
    assert ref.status == 0 and min(ref.active_hist) < 8
    ctx = upload(A, False)
    ctx.set_precond_offset(4.0)
    ctx.set_soft_lock(True)
    X = to_dev(W.initial_block(A.n, 8, seed=1), np.float64)
    r = ctx.solve(X, 5, history=True, maxiter=200)
    assert r.status == 0 and r.locked_max == 8 - min(ref.active_hist), (r.locked_max, ref.active_hist)
    th, ref_th = r.theta_hist, np.array(ref.theta_hist)
    m = min(len(th), len(ref_th))
    print(f"{len(th)} GPU / {len(ref_th)} oracle iterations, active widths {ref.active_hist}")
    assert m >= 3 and abs(len(th) - len(ref_th)) <= 1
    np.testing.assert_allclose(th[:m], ref_th[:m], rtol=1e-9)
