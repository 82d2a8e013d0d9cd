"""GPU parity of the individual hot-path kernels against the FP64 oracle,
called through the C ABI (ctypes binding).

Bars: bitwise for integer-valued inputs (any summation order is exact there,
so a race or a lost atomic update shows up as a mismatch); FP32 SpMM within
1e-5 of the condition-aware row scale ||(|H||X|)_i||, and within 1e-5 of
||(HX)_i|| on every row whose terms do not cancel below 1e-2 of that scale;
FP64 within 1e-12 of the first and 1e-10 of the second.
"""
import numpy as np
import pytest

import oracle
import synth
from synth import workloads as W
from gpu_util import row_error, torch_cuda, to_dev, upload

pytestmark = pytest.mark.gpu


def int_matrix(n, draws, seed, vmax=4, hubs=False):
    """random_sym (or power-law, with rows longer than the CSR kernel's
    one-workgroup threshold) pattern with small integer values (exact in FP32
    and BF16)."""
    A = synth.zipf(n, lmin=4, lmax=6000, seed=seed) if hubs else synth.random_sym(n, draws, seed=seed, f32=False)
    rng = np.random.default_rng(seed)
    v = rng.integers(-vmax, vmax + 1, size=A.nnz).astype(np.float64)
    v[v == 0] = 1.0
    diag_pos = A.row_ptr[:-1]
    v[diag_pos] = rng.integers(0, 9, size=A.n)
    return synth.ArrayCSR(A.n, A.row_ptr.copy(), A.col.copy(), v)


MATRICES = {
    "random_sym": lambda: synth.random_sym(3000, 20, seed=3),
    "tiled": lambda: synth.tiled(64 * 40, tile=64, tile_draws=5, p=0.1, seed=2),
    "zipf": lambda: synth.zipf(4000, lmin=4, lmax=400, seed=5),
    "tiny": lambda: synth.random_sym(7, 3, seed=1),
    # power-law rows: ~270 of them longer than 1024 entries (the CSR long-row kernel)
    "hubs": lambda: synth.zipf(20000, lmin=4, lmax=6000, seed=7),
}


@pytest.mark.parametrize("name", list(MATRICES))
@pytest.mark.parametrize("k", [1, 4, 5, 8, 16])
@pytest.mark.parametrize("f32", [True, False])
@pytest.mark.parametrize("fmt", ["csr", "tiled"])
def test_spmm_parity(name, k, f32, fmt):
    import paper_2109_00485_amd as L
    torch = torch_cuda()
    A = MATRICES[name]()
    dt = np.float32 if f32 else np.float64
    ctx = upload(A, f32, fmt={"csr": L.FORMAT_CSR, "tiled": L.FORMAT_TILED}[fmt])
    assert ctx.query()["format"] == (L.FORMAT_CSR if fmt == "csr" else L.FORMAT_TILED)
    X = synth.gaussian_block(A.n, k, seed=17).astype(dt)
    Y = ctx.spmm_sym(to_dev(X, dt)).cpu().numpy()
    H = oracle.SymMatrix(A.n, A.row_ptr, A.col, np.asarray(A.val, dtype=dt))
    Yref = H @ X.astype(np.float64)
    Yabs = H.abs_matmul(X.astype(np.float64))
    err = row_error(Y, Yref, Yabs)
    assert err <= (1e-5 if f32 else 1e-12), err
    # the relative row-norm error against ||(HX)_i|| itself, on the rows whose
    # terms do not cancel to below 1e-2 of ||(|H||X|)_i|| (those are counted;
    # at k >= 4 there are none in these matrices, at k = 1 at most 11 rows)
    num = np.linalg.norm(np.asarray(Y, dtype=np.float64) - Yref, axis=1)
    den = np.linalg.norm(Yref, axis=1)
    keep = den > 1e-2 * np.linalg.norm(Yabs, axis=1)
    rel = float(np.max(num[keep] / den[keep])) if np.any(keep) else 0.0
    print(f"{name} k={k} f32={f32} {fmt}: |H||X| scale {err:.2e}, ||HX|| scale {rel:.2e} "
          f"({np.count_nonzero(~keep)} of {A.n} rows cancel below 1e-2)")
    assert rel <= (1e-5 if f32 else 1e-10), rel


@pytest.mark.parametrize("k", [1, 4, 8, 16])
@pytest.mark.parametrize("fmt", ["csr", "tiled"])
@pytest.mark.parametrize("hubs", [False, True])
def test_spmm_integer_bitwise(k, fmt, hubs):
    import paper_2109_00485_amd as L
    torch = torch_cuda()
    A = int_matrix(20000 if hubs else 2000, 25, seed=4, hubs=hubs)
    ctx = upload(A, True, fmt={"csr": L.FORMAT_CSR, "tiled": L.FORMAT_TILED}[fmt])
    X = np.random.default_rng(0).integers(-8, 9, size=(A.n, k)).astype(np.float32)
    Y = ctx.spmm_sym(to_dev(X, np.float32)).cpu().numpy()
    Yref = oracle.SymMatrix(A.n, A.row_ptr, A.col, A.val) @ X
    assert np.array_equal(Y.astype(np.float64), Yref)


def test_format_choice():
    """AUTO picks the tiled format when the stored entries fill the 64 x 64
    tiles they touch densely enough (at least 64 entries per touched tile on
    average), 32-bit CSR indices otherwise; a forced tiled format works on the
    sparse-tiled matrix too.  Both give the oracle's rows."""
    import paper_2109_00485_amd as L
    torch = torch_cuda()
    A = synth.tiled(64 * 200, tile_draws=20, p=0.05, seed=3)
    assert upload(A, True).query()["format"] == L.FORMAT_TILED
    # ~20 entries per touched tile: the CSR product is the faster one there
    assert upload(W.make_matrix("random_sym_20k"), False).query()["format"] == L.FORMAT_CSR
    B = synth.random_sym(200_000, 50, seed=3, f32=True)   # ~1 entry per touched tile
    H = oracle.SymMatrix.from_csr(B)
    X = synth.gaussian_block(B.n, 8, seed=2).astype(np.float32)
    rows = np.random.default_rng(0).choice(B.n, 2000, replace=False)
    Yr, Ya = H.rows(X.astype(np.float64), rows)
    for fmt, want in ((None, L.FORMAT_CSR), (L.FORMAT_TILED, L.FORMAT_TILED)):
        ctx = upload(B, True, fmt=fmt)
        assert ctx.query()["format"] == want
        Y = ctx.spmm_sym(to_dev(X, np.float32)).cpu().numpy()
        assert row_error(Y[rows], Yr, Ya) <= 1e-5
        ctx.close()


def test_spmm_repeatable_and_no_alias():
    import paper_2109_00485_amd as L
    torch = torch_cuda()
    A = int_matrix(1500, 30, seed=6)
    ctx = upload(A, True)
    X = to_dev(np.random.default_rng(1).integers(-8, 9, size=(A.n, 8)), np.float32)
    Y1 = ctx.spmm_sym(X).cpu()
    Y2 = ctx.spmm_sym(X).cpu()
    assert torch.equal(Y1, Y2)
    with pytest.raises(L.LobpcgError):
        ctx.spmm_sym(X, X)
    with pytest.raises(L.LobpcgError):
        ctx.spmm_sym(to_dev(np.zeros((A.n, 17)), np.float32))


@pytest.mark.parametrize("ka,kb", [(8, 8), (5, 13), (24, 48), (48, 48), (1, 1)])
@pytest.mark.parametrize("prec", ["f64", "f32", "bf16x3", "bf16x6", "f64ctx"])
def test_gram_parity(ka, kb, prec):
    import paper_2109_00485_amd as L
    torch = torch_cuda()
    n = 5003  # several slabs of 16 rows, ragged tail
    A = synth.random_sym(n, 2, seed=1)
    f32 = prec != "f64ctx"
    dt = np.float32 if f32 else np.float64
    ctx = upload(A, f32)
    a = synth.gaussian_block(n, ka, seed=2).astype(dt)
    b = synth.gaussian_block(n, kb, seed=3).astype(dt)
    p = {"f64": L.GRAM_F64, "f32": L.GRAM_F32, "bf16x3": L.GRAM_BF16X3, "bf16x6": L.GRAM_BF16X6,
         "f64ctx": L.GRAM_F64}[prec]
    G = ctx.gram(to_dev(a, dt), to_dev(b, dt), prec=p).cpu().numpy()
    ref = a.astype(np.float64).T @ b.astype(np.float64)
    scale = np.sqrt(np.outer((a.astype(np.float64) ** 2).sum(0), (b.astype(np.float64) ** 2).sum(0)))
    # bf16x6: dropped products below 2^-24 relative, FP32 sums of 16 rows (~2^-24 each)
    tol = {"f64": 1e-13, "f64ctx": 1e-13, "f32": 2e-6, "bf16x3": 2e-5, "bf16x6": 2e-7}[prec]
    err = np.max(np.abs(G - ref) / scale)
    assert err <= tol, err


@pytest.mark.parametrize("k", [5, 8, 16, 24])
@pytest.mark.parametrize("prec", ["f64", "f32", "bf16x6", "f64ctx"])
def test_gram_same_block_parity(k, prec):
    """A^T A with the same block on both sides (the kernel loads it once and
    uses it as both operands; one 16-column tile for k <= 16, two for k = 24)
    against the FP64 product.  With one product per entry pair (FP64, FP32)
    the result is exactly symmetric; the split-BF16 terms of (i, j) and (j, i)
    are summed in different orders."""
    import paper_2109_00485_amd as L
    torch_cuda()
    n = 4099
    A = synth.random_sym(n, 2, seed=1)
    f32 = prec != "f64ctx"
    dt = np.float32 if f32 else np.float64
    ctx = upload(A, f32)
    a = synth.gaussian_block(n, k, seed=6).astype(dt)
    p = {"f64": L.GRAM_F64, "f32": L.GRAM_F32, "bf16x6": L.GRAM_BF16X6, "f64ctx": L.GRAM_F64}[prec]
    ad = to_dev(a, dt)
    G = ctx.gram(ad, ad, prec=p).cpu().numpy()
    ref = a.astype(np.float64).T @ a.astype(np.float64)
    scale = np.sqrt(np.outer(np.diag(ref), np.diag(ref)))
    tol = {"f64": 1e-13, "f64ctx": 1e-13, "f32": 2e-6, "bf16x6": 2e-7}[prec]
    assert np.max(np.abs(G - ref) / scale) <= tol
    if prec != "bf16x6":
        assert np.array_equal(G, G.T)


@pytest.mark.parametrize("prec", ["f64", "f32", "bf16x3", "bf16x6"])
def test_gram_integer_exact(prec):
    import paper_2109_00485_amd as L
    torch = torch_cuda()
    n = 1111
    A = synth.random_sym(n, 2, seed=1)
    ctx = upload(A, True)
    rng = np.random.default_rng(5)
    a = rng.integers(-16, 17, size=(n, 24)).astype(np.float32)
    b = rng.integers(-16, 17, size=(n, 48)).astype(np.float32)
    p = {"f64": L.GRAM_F64, "f32": L.GRAM_F32, "bf16x3": L.GRAM_BF16X3, "bf16x6": L.GRAM_BF16X6}[prec]
    G = ctx.gram(to_dev(a, np.float32), to_dev(b, np.float32), prec=p).cpu().numpy()
    assert np.array_equal(G, a.astype(np.float64).T @ b.astype(np.float64))


@pytest.mark.parametrize("offset", [0.0, 2.5])
@pytest.mark.parametrize("f32", [True, False])
def test_precond_diag_parity(f32, offset):
    import paper_2109_00485_amd as L
    from oracle.precond import diag_precond
    torch = torch_cuda()
    A = synth.random_sym(2000, 10, seed=8, f32=f32)
    dt = np.float32 if f32 else np.float64
    ctx = upload(A, f32)
    ctx.set_precond_offset(offset)
    gamma = ctx.query()["gamma"]
    R = synth.gaussian_block(A.n, 8, seed=4).astype(dt)
    # shifts chosen so that some d_i - theta_j fall inside the guard band
    theta = np.array([A.diag[0], A.diag[10], -1.0, 5.0, A.diag[100] + 1e-9, 0.0, 100.0, A.diag[-1]])
    W = ctx.precond_apply(to_dev(R, dt), to_dev(theta, np.float64), kind=L.PRECOND_DIAG).cpu().numpy()
    ref = diag_precond(R.astype(np.float64), np.asarray(A.diag, dtype=dt).astype(np.float64), theta, 1e-5 * gamma,
                       offset=offset)
    rtol = 1e-6 if f32 else 1e-15
    np.testing.assert_allclose(W, ref, rtol=rtol)
    Wn = ctx.precond_apply(to_dev(R, dt), to_dev(theta, np.float64), kind=L.PRECOND_NONE).cpu().numpy()
    assert np.array_equal(Wn, R)


def test_gershgorin_matches_oracle():
    torch = torch_cuda()
    A = synth.zipf(3000, lmin=4, lmax=300, seed=3, f32=False)
    ctx = upload(A, False)
    H = oracle.SymMatrix.from_csr(A)
    assert ctx.query()["gamma"] == pytest.approx(H.gershgorin(), rel=1e-13)
    d = ctx.diag().cpu().numpy()
    assert np.array_equal(d, A.diag)


@pytest.mark.parametrize("fmt", ["csr", "tiled"])
def test_row_statistics_deterministic(fmt):
    """gamma and the per-row network features (full-row off-diagonal 1-norm,
    mean |h| of the row's 64-row tile) are the same bits in every context and
    match the oracle's definitions (a power-law pattern, hubs included, and a
    ragged last tile)."""
    import paper_2109_00485_amd as L
    torch = torch_cuda()
    if fmt == "csr":
        A = synth.zipf(20000 + 37, lmin=4, lmax=3000, seed=11, f32=False)
    else:
        A = synth.tiled(64 * 60, tile=64, tile_draws=5, p=0.1, seed=2)
    H = oracle.SymMatrix.from_csr(A)
    f = {"csr": L.FORMAT_CSR, "tiled": L.FORMAT_TILED}[fmt]
    runs = []
    for _ in range(3):
        ctx = upload(A, False, fmt=f)
        rho, tm = (x.cpu().numpy() for x in ctx.features())
        runs.append((ctx.query()["gamma"], rho, tm))
        ctx.close()
    for g, rho, tm in runs[1:]:
        assert g == runs[0][0] and np.array_equal(rho, runs[0][1]) and np.array_equal(tm, runs[0][2])
    g, rho, tm = runs[0]
    assert g == pytest.approx(H.gershgorin(), rel=1e-13)
    off = H.row_offdiag_abs()
    np.testing.assert_allclose(rho, off.astype(np.float32), rtol=1e-6)
    cnt = H.row_offdiag_count().astype(np.float64)
    nt = (A.n + 63) // 64
    pad = nt * 64 - A.n
    tile_mean = (np.concatenate([off, np.zeros(pad)]).reshape(nt, 64).sum(1) /
                 np.maximum(np.concatenate([cnt, np.zeros(pad)]).reshape(nt, 64).sum(1), 1))
    np.testing.assert_allclose(tm, np.repeat(tile_mean, 64)[:A.n].astype(np.float32), rtol=1e-6)


def test_create_rejects_malformed():
    import paper_2109_00485_amd as L
    torch = torch_cuda()
    A = synth.random_sym(500, 5, seed=2, f32=False)

    def try_create(rp, col, val):
        class _A:
            pass
        a = _A()
        a.n, a.row_ptr, a.col, a.val = A.n, rp, col, val
        return L.Context.from_csr(a, dtype=L.F64)
    # lower-triangle entry
    col = A.col.copy()
    col[A.row_ptr[10] + 1] = 3
    with pytest.raises(L.LobpcgError) as e:
        try_create(A.row_ptr, col, A.val)
    assert e.value.status == L.EINVAL
    # missing diagonal (first entry of row 20 replaced by its successor's column)
    col = A.col.copy()
    col[A.row_ptr[20]] = col[A.row_ptr[20] + 1] - 0 if A.row_ptr[21] - A.row_ptr[20] > 1 else 499
    with pytest.raises(L.LobpcgError):
        try_create(A.row_ptr, col, A.val)
    # out-of-range column
    col = A.col.copy()
    col[A.row_ptr[5] + 1] = A.n + 7
    with pytest.raises(L.LobpcgError):
        try_create(A.row_ptr, col, A.val)
    # row_ptr beyond nnz (must be rejected without reading out of bounds)
    rp = A.row_ptr.copy()
    rp[100] = A.nnz + 1000
    with pytest.raises(L.LobpcgError):
        try_create(rp, A.col, A.val)
    # NaN value
    val = A.val.copy()
    val[17] = np.nan
    with pytest.raises(L.LobpcgError) as e:
        try_create(A.row_ptr, A.col, val)
    assert e.value.status == L.ENONFINITE


@pytest.mark.parametrize("fmt", ["csr", "tiled"])
def test_create_with_int32_row_offsets(fmt):
    """lobpcg_create_rp32: int32 row offsets give the same context as int64 ones
    (bitwise the same product), and malformed int32 offsets are rejected."""
    import paper_2109_00485_amd as L
    torch = torch_cuda()
    A = synth.tiled(64 * 30, tile=64, tile_draws=5, p=0.1, seed=2) if fmt == "tiled" else \
        synth.random_sym(3000, 20, seed=3)

    class _A:
        pass
    a = _A()
    a.n, a.row_ptr, a.col, a.val = A.n, A.row_ptr.astype(np.int32), A.col, np.asarray(A.val, dtype=np.float32)
    f = {"csr": L.FORMAT_CSR, "tiled": L.FORMAT_TILED}[fmt]
    c32 = L.Context.from_csr(a, dtype=L.F32, fmt=f)
    c64 = upload(A, True, fmt=f)
    assert c32.query() == c64.query()
    X = to_dev(synth.gaussian_block(A.n, 8, seed=4).astype(np.float32), np.float32)
    assert torch.equal(c32.spmm_sym(X), c64.spmm_sym(X))
    rp = A.row_ptr.astype(np.int32)
    rp[50] = rp[49] - 1     # decreasing offsets
    a.row_ptr = rp
    with pytest.raises(L.LobpcgError) as e:
        L.Context.from_csr(a, dtype=L.F32, fmt=f)
    assert e.value.status == L.EINVAL
