"""GPU block-diagonal FOM preconditioner (LOBPCG_PRECOND_FOM, Section 3.4)
against the FP64 oracle (oracle.precond.block_fom_precond on the diagonal
tiles the oracle builds itself from the upper-triangle CSR).

Both sides run FOM in FP64 on the same inputs (FP32 contexts: the FP32 matrix
values and block, upcast exactly), so they differ by rounding order only.  The
bar is per (tile, column) block, relative to the block's largest entry: 1e-9
in FP64 and 1e-6 in FP32 (there the output itself is rounded to FP32), raised
where the oracle's own iterate is sensitive to rounding: each block is also
solved by the oracle with its right-hand side perturbed by 1e-13 (relative,
twice), and the bar becomes 1e-2 of the change that caused (an iterate whose
H_m is nearly singular amplifies rounding; the perturbation is 1e3 units in
the last place, the GPU's rounding differences a few).  Where the perturbed
solves disagree on whether a FOM iterate exists at all (the singularity or
breakdown test decided by rounding), both answers are correct: the GPU block
must then be one of the oracle's iterates or the guarded diagonal step.  Such
blocks are rare (a ragged tail tile whose diagonal entries cluster), and the
tests bound how many there may be.
"""
import numpy as np
import pytest

import oracle
import synth
from gpu_util import torch_cuda, to_dev, upload
from oracle.lobpcg import lobpcg as oracle_lobpcg
from oracle.precond import block_fom_precond, diag_precond, diagonal_tiles, fom, guard, shifts
from synth import workloads as W

pytestmark = pytest.mark.gpu

MATRICES = {
    # full 64-row tiles with a block-sparse pattern
    "tiled": lambda f32: synth.tiled(64 * 40, tile=64, tile_draws=5, p=0.1, seed=2, f32=f32),
    # a ragged last tile (n = 30 * 64 + 17)
    "random_sym": lambda f32: synth.random_sym(64 * 30 + 17, 12, seed=9, f32=f32),
    # dense tiles: every entry of each diagonal tile present, ragged tail of 22 rows
    "dense": lambda f32: synth.from_dense_upper(_dense_sym(150, seed=4), dtype=np.float32 if f32 else np.float64),
}


def _dense_sym(n, seed):
    rng = np.random.default_rng(seed)
    B = rng.standard_normal((n, n)) * 0.3
    return 0.5 * (B + B.T) + np.diag(np.linspace(1.0, 40.0, n))


def _check_against_oracle(Wg, tiles, R, theta, m, eps, offset, n, floor):
    """Compare the GPU block Wg with the oracle block by block (see the module
    docstring); returns the number of blocks decided by rounding."""
    ref = block_fom_precond(tiles, R, theta, m, eps, offset=offset)
    sig = shifts(theta, offset)
    rng = np.random.default_rng(123)
    k = R.shape[1]
    T = tiles.shape[1]
    ambiguous = 0
    for t in range(tiles.shape[0]):
        lo, hi = t * T, min(n, (t + 1) * T)
        for j in range(k):
            b = np.zeros(T)
            b[:hi - lo] = R[lo:hi, j]
            Kj = tiles[t] - sig[j] * np.eye(T)
            x0, ok0 = fom(Kj, b, m)
            runs = [fom(Kj, b * (1.0 + 1e-13 * rng.standard_normal(T)), m) for _ in range(2)]
            g, r = Wg[lo:hi, j], ref[lo:hi, j]
            scale = np.abs(r).max()
            if scale == 0.0:
                assert np.all(g == 0.0), (t, j)
                continue
            if all(ok == ok0 for _, ok in runs):
                dev = max(np.abs(x[:hi - lo] - x0[:hi - lo]).max() for x, _ in runs) / scale
                err = np.abs(g - r).max() / scale
                assert err <= max(floor, 1e-2 * dev), (t, j, err, dev)
            else:
                ambiguous += 1
                cands = [x[:hi - lo] for x, ok in [(x0, ok0)] + runs if ok]
                cands.append(R[lo:hi, j] / guard(np.diag(tiles[t])[:hi - lo] - sig[j], eps))
                errs = [np.abs(g - c).max() / max(np.abs(c).max(), 1e-300) for c in cands]
                assert min(errs) <= max(floor, 1e-6), (t, j, errs)
    return ambiguous


def _theta_for(A, k, seed):
    """Shifts spread over the diagonal's range, some at diagonal entries."""
    d = np.asarray(A.diag, dtype=np.float64)
    rng = np.random.default_rng(seed)
    th = np.sort(rng.uniform(d.min(), d.max(), size=k))
    th[0] = d[3]
    return th


@pytest.mark.parametrize("name", list(MATRICES))
@pytest.mark.parametrize("f32", [False, True])
@pytest.mark.parametrize("m", [1, 2, 4, 8])
@pytest.mark.parametrize("offset", [0.0, 2.5])
def test_fom_apply_parity(name, f32, m, offset):
    import paper_2109_00485_amd as L
    torch_cuda()
    A = MATRICES[name](f32)
    dt = np.float32 if f32 else np.float64
    ctx = upload(A, f32)
    ctx.set_precond_offset(offset)
    ctx.set_fom_steps(m)
    gamma = ctx.query()["gamma"]
    k = 8
    R = synth.gaussian_block(A.n, k, seed=5).astype(dt)
    theta = _theta_for(A, k, seed=m)
    Wg = ctx.precond_apply(to_dev(R, dt), to_dev(theta, np.float64), kind=L.PRECOND_FOM).cpu().numpy()
    tiles = diagonal_tiles(A.n, A.row_ptr, A.col, np.asarray(A.val, dtype=dt).astype(np.float64))
    amb = _check_against_oracle(Wg.astype(np.float64), tiles, R.astype(np.float64), theta, m, 1e-5 * gamma, offset,
                                A.n, 1e-6 if f32 else 1e-9)
    assert amb <= 0.02 * k * tiles.shape[0], amb


@pytest.mark.parametrize("k", [1, 5, 16])
def test_fom_block_widths(k):
    """Columns c = wave, wave + 4, ...: widths below, between and above the
    four waves of a workgroup."""
    import paper_2109_00485_amd as L
    torch_cuda()
    A = MATRICES["random_sym"](False)
    ctx = upload(A, False)
    gamma = ctx.query()["gamma"]
    R = synth.gaussian_block(A.n, k, seed=6)
    theta = _theta_for(A, k, seed=1) if k > 1 else np.array([float(A.diag[3])])
    Wg = ctx.precond_apply(to_dev(R, np.float64), to_dev(theta, np.float64), kind=L.PRECOND_FOM).cpu().numpy()
    tiles = diagonal_tiles(A.n, A.row_ptr, A.col, A.val)
    assert _check_against_oracle(Wg, tiles, R, theta, 4, 1e-5 * gamma, 0.0, A.n, 1e-9) <= 0.02 * k * tiles.shape[0]


def test_fom_diagonal_matrix_invariant_space_and_singular_tile():
    """A diagonal H: each tile is diagonal, so the Krylov space of a right-hand
    side with s <= m nonzeros in a tile is invariant after s steps and FOM is
    the exact solve, i.e. the diagonal step R_ij / (d_i - sigma_j).  A column
    whose shift equals d_i and whose right-hand side in that tile is e_i gives
    the zero 1 x 1 Hessenberg: no FOM iterate, the guarded step R_ij / eps."""
    import paper_2109_00485_amd as L
    torch_cuda()
    n, k = 64 * 6 + 9, 4
    d = np.linspace(1.0, 50.0, n)
    A = synth.diagonal(d)
    ctx = upload(A, False)
    gamma = ctx.query()["gamma"]
    eps = 1e-5 * gamma
    rng = np.random.default_rng(2)
    R = np.zeros((n, k))
    for lo in range(0, n, 64):
        hi = min(n, lo + 64)
        for j in range(k):
            rows = rng.choice(np.arange(lo, hi), size=min(3, hi - lo), replace=False)
            R[rows, j] = rng.standard_normal(rows.size)
    # column 2 of tile 1: right-hand side e_70 with sigma = d_70
    R[64:128, 2] = 0.0
    R[70, 2] = 1.0
    theta = np.array([0.5, 20.25, d[70], 60.0])
    Wg = ctx.precond_apply(to_dev(R, np.float64), to_dev(theta, np.float64), kind=L.PRECOND_FOM).cpu().numpy()
    ref = diag_precond(R, d, theta, eps)
    np.testing.assert_allclose(Wg, ref, rtol=1e-12, atol=0)
    assert Wg[70, 2] == pytest.approx(1.0 / eps, rel=1e-15)


def test_fom_steps_validation_and_default():
    import paper_2109_00485_amd as L
    torch_cuda()
    A = MATRICES["random_sym"](False)
    ctx = upload(A, False)
    for bad in (0, 9, -1):
        with pytest.raises(L.LobpcgError):
            ctx.set_fom_steps(bad)
    # the default is 4 steps
    gamma = ctx.query()["gamma"]
    R = synth.gaussian_block(A.n, 8, seed=7)
    theta = _theta_for(A, 8, seed=3)
    W4 = ctx.precond_apply(to_dev(R, np.float64), to_dev(theta, np.float64), kind=L.PRECOND_FOM).cpu().numpy()
    tiles = diagonal_tiles(A.n, A.row_ptr, A.col, A.val)
    assert _check_against_oracle(W4, tiles, R, theta, 4, 1e-5 * gamma, 0.0, A.n, 1e-9) <= 0.02 * 8 * tiles.shape[0]


@pytest.mark.parametrize("f32", [False, True])
def test_fom_solve_against_oracle(f32):
    """LOBPCG with the block-diagonal FOM preconditioner (shift at theta_j,
    m = 2) on a 64-tiled matrix: the same eigenvalues as the oracle's LOBPCG
    with the oracle's FOM preconditioner.  The iteration counts depend on
    rounding (with the shift at theta_j the diagonal step is nearly singular)
    and are printed, not compared; the next test compares them over starts."""
    import paper_2109_00485_amd as L
    A = MATRICES["tiled"](f32)
    H = oracle.SymMatrix.from_csr(A)
    tiles = diagonal_tiles(A.n, A.row_ptr, A.col, A.val)
    eps = 1e-5 * H.gershgorin()
    X0 = W.initial_block(A.n, 8, seed=1)
    ref = oracle_lobpcg(H, X0, 5, precond=lambda R, th, X: block_fom_precond(tiles, R, th, 2, eps), maxiter=3000)
    ctx = upload(A, f32)
    dt = np.float32 if f32 else np.float64
    r_diag = ctx.solve(to_dev(X0, dt), 5, maxiter=3000)
    ctx.set_fom_steps(2)
    X = to_dev(X0, dt)
    r = ctx.solve(X, 5, maxiter=3000, precond=L.PRECOND_FOM)
    assert r.status == 0 and r_diag.status == 0, (r, r_diag)
    print(f"iterations: diagonal {r_diag.iters}, FOM m=2 {r.iters} (oracle FOM {ref.iters})")
    lam = ref.theta
    tau = 1e-3 * H.gershgorin()
    assert np.all(np.abs(r.evals[:5] - lam) <= 1e-6 * np.maximum(np.abs(lam), tau)), (r.evals[:5], lam)
    Xg = X.cpu().numpy().astype(np.float64)
    G = Xg.T @ Xg
    assert np.abs(G - np.eye(8)).max() < (2e-5 if f32 else 1e-10)


def test_fom_fewer_iterations_over_starts():
    """The FOM preconditioner against the diagonal step at the same shift
    (theta_j, m = 2), FP64, from six Gaussian starts: fewer iterations on
    average.  One start alone says little: with the shift at theta_j the
    diagonal step is nearly singular and a single count moves by a factor of
    up to 3 with the rounding of the trajectory."""
    import paper_2109_00485_amd as L
    A = MATRICES["tiled"](False)
    ctx = upload(A, False)
    ctx.set_fom_steps(2)
    its = {"diag": [], "fom": []}
    for seed in range(1, 7):
        for name, pc in (("diag", L.PRECOND_DIAG), ("fom", L.PRECOND_FOM)):
            r = ctx.solve(to_dev(W.initial_block(A.n, 8, seed=seed), np.float64), 5, maxiter=3000, precond=pc)
            assert r.status == 0, (name, seed, r.status)
            its[name].append(r.iters)
    print("iterations", its)
    assert np.mean(its["fom"]) < 0.8 * np.mean(its["diag"]), its
