"""The solve's orthogonalisation step (Section 3.5; Algorithm 1 before the
product H W) through lobpcg_orthonormalize, against the FP64 oracle's two
steps, W - X (X^T W) followed by oracle.dense.cholqr.

The GPU forms the projected block's Gram from one Gram of [X W]
(W^T W - C^T C - C^T C + C^T (X^T X) C with C = X^T W) and writes
W R^{-1} - X (C R^{-1}) in one pass; in exact arithmetic this is the oracle's
Q, which is unique (the Q of a QR factorisation whose R has a positive
diagonal), so the two are compared entry by entry.  Bars: FP64 1e-13 (the
projected blocks here have condition numbers below 1e2 and column ratios
||w_j|| / ||w_j - X C_j|| up to ~5, like the solves'; 6.4e-16 measured); FP32
contexts 1e-6 on the FP32-rounded inputs (6.5e-8 measured: the output's own
rounding; X then is not exactly orthonormal, and the formula is exact for any
X, as is the oracle's projection)."""
import numpy as np
import pytest

from gpu_util import to_dev, torch_cuda, upload
from oracle.dense import NotSPD, cholqr
from synth import workloads as W

pytestmark = pytest.mark.gpu


def blocks(n, k, seed, mix=3.0):
    """X orthonormal; W with an X component `mix` times its own part."""
    rng = np.random.default_rng(seed)
    X, _ = np.linalg.qr(rng.standard_normal((n, k)))
    Wm = rng.standard_normal((n, k)) + X @ (mix * np.sqrt(n / k) * rng.standard_normal((k, k)))
    return X, Wm


def oracle_q(X, Wm):
    return cholqr(Wm - X @ (X.T @ Wm))[0]


@pytest.mark.parametrize("f32", [False, True])
@pytest.mark.parametrize("k", [1, 5, 8, 16])
def test_orthonormalize_against_oracle(f32, k):
    torch_cuda()
    A = W.make_matrix("random_sym_1k")   # n = 1000: a ragged last 16-row slab
    ctx = upload(A, f32)
    dt = np.float32 if f32 else np.float64
    X, Wm = blocks(A.n, k, seed=k)
    X, Wm = X.astype(dt).astype(np.float64), Wm.astype(dt).astype(np.float64)
    Q = to_dev(Wm, dt)
    assert ctx.orthonormalize(to_dev(X, dt), Q) == 0
    Qg = Q.cpu().numpy().astype(np.float64)
    Qr = oracle_q(X, Wm)
    ratio = np.linalg.norm(Wm, axis=0) / np.linalg.norm(Wm - X @ (X.T @ Wm), axis=0)
    err = np.abs(Qg - Qr).max()
    print(f"k={k} f32={f32}: max |Q - Q_oracle| {err:.2e}, column ratio up to {ratio.max():.1f}, "
          f"|X^T Q| {np.abs(X.T @ Qg).max():.2e}, |Q^T Q - I| {np.abs(Qg.T @ Qg - np.eye(k)).max():.2e}")
    assert err <= (1e-6 if f32 else 1e-13), err


def test_orthonormalize_large_n_fp32():
    """n = 2e6 FP32 (the bench's block size), k = 8: orthonormal and orthogonal
    to X to FP32 rounding, and on 4096 sampled rows equal to the oracle's Q
    (the oracle's factor from its own full FP64 Gram)."""
    torch = torch_cuda()
    n, k = 2_000_000, 8
    rng = np.random.default_rng(7)
    X, _ = np.linalg.qr(rng.standard_normal((n, k)))
    Wm = rng.standard_normal((n, k)) + X @ (3.0 * np.sqrt(n / k) * rng.standard_normal((k, k)))
    X, Wm = X.astype(np.float32).astype(np.float64), Wm.astype(np.float32).astype(np.float64)
    import synth
    ctx = upload(synth.diagonal(np.linspace(1.0, 2.0, n)), True)
    Q = to_dev(Wm, np.float32)
    assert ctx.orthonormalize(to_dev(X, np.float32), Q) == 0
    Qg = Q.cpu().numpy().astype(np.float64)
    assert np.abs(Qg.T @ Qg - np.eye(k)).max() < 1e-5
    assert np.abs(X.T @ Qg).max() < 1e-5
    Qr = oracle_q(X, Wm)
    rows = rng.choice(n, 4096, replace=False)
    assert np.abs(Qg[rows] - Qr[rows]).max() < 2e-5


def test_orthonormalize_column_in_span_of_x():
    """A column of W equal to a column of X (exactly orthonormal X of unit
    vectors): its projection is exactly zero, the Gram is singular, the call
    returns LOBPCG_ENOTSPD and leaves W unchanged; the oracle raises on the same
    blocks."""
    import paper_2109_00485_amd as L
    torch_cuda()
    A = W.make_matrix("random_sym_1k")
    ctx = upload(A, False)
    n, k = A.n, 8
    X = np.zeros((n, k))
    X[np.arange(k) * 7, np.arange(k)] = 1.0
    rng = np.random.default_rng(1)
    Wm = rng.standard_normal((n, k))
    Wm[:, 3] = X[:, 0]
    Q = to_dev(Wm, np.float64)
    with pytest.raises(L.LobpcgError) as e:
        ctx.orthonormalize(to_dev(X, np.float64), Q)
    assert e.value.status == L.ENOTSPD
    assert np.array_equal(Q.cpu().numpy(), Wm)
    with pytest.raises(NotSPD):
        oracle_q(X, Wm)


def test_orthonormalize_validation():
    """k above the context's block width bound (16) is rejected before any launch."""
    import paper_2109_00485_amd as L
    torch_cuda()
    ctx = upload(W.make_matrix("random_sym_1k"), False)
    X = to_dev(np.zeros((1000, 17)), np.float64)
    Wm = to_dev(np.ones((1000, 17)), np.float64)
    with pytest.raises(L.LobpcgError) as e:
        ctx.orthonormalize(X, Wm)
    assert e.value.status == L.EINVAL
