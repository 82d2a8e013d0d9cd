"""Learned preconditioner on the GPU against the FP64 oracle (oracle.mlp,
oracle.harvest): the matrix-core forward pass, the preconditioner apply, the
group loss and its gradient, one Adam step, the standardiser, the harvest of
training samples, and solves with an attached network.

Tolerances.  The network's BF16 rounding of the first hidden layer is taken in
FP32 on both sides (oracle ``a1_f32``); the rest of the oracle is FP64 and the
kernels accumulate in FP32, so outputs agree to ~1e-5 of the output's
magnitude scale  S = sum_v |w3_v| (|b2_v| + sum_u |W2_vu| |h1_u|) + |b3|.
A different summation order can still move a first-layer value across a BF16
rounding boundary; such a flip changes o by at most 2^-8 S, and is allowed for
a small fraction of samples.  Gradients carry the FP32 accumulation error of
sums over the batch: 1e-4 relative per parameter block.
"""
import numpy as np
import pytest

from gpu_util import to_dev, torch_cuda, upload
from oracle import harvest as OH
from oracle import mlp as OM
from synth import workloads as W

pytestmark = pytest.mark.gpu


def params(seed, mu=(100.0, -1.0, 30.0, 0.4), sigma=(50.0, 0.5, 5.0, 0.1), scale3=0.1):
    p = OM.init_params(seed, mu=list(mu), sigma=list(sigma))
    rng = np.random.default_rng(seed + 100)
    p.w3 = rng.standard_normal(64) * scale3
    p.b1 = rng.standard_normal(64) * 0.1
    p.b2 = rng.standard_normal(64) * 0.1
    p.b3 = 0.05
    return p


def blob(p):
    import paper_2109_00485_amd as L
    return L.pack_params(dict(W1=p.W1, b1=p.b1, W2=p.W2, b2=p.b2, w3=p.w3, b3=p.b3, mu=p.mu, sigma=p.sigma))


def as_f32_params(p):
    """The oracle parameters as the device holds them (FP32 master weights)."""
    q = p.copy()
    for key in ("W1", "b1", "W2", "b2", "w3", "mu", "sigma"):
        setattr(q, key, np.asarray(getattr(p, key), dtype=np.float32).astype(np.float64))
    q.b3 = float(np.float32(p.b3))
    return q


def scale_of(p, z):
    o, (z, a1, h1b, a2, h2, W1b, W2b, w3b) = OM.forward(p, z, a1_f32=True)
    S = np.abs(w3b) @ (np.abs(p.b2)[:, None] + np.abs(W2b) @ np.abs(h1b).T) + abs(p.b3)
    return o, S


def features(rng, N):
    return np.column_stack([rng.uniform(0, 200, N), rng.uniform(-3, 1, N), rng.uniform(20, 45, N),
                            rng.uniform(0.3, 0.5, N)])


def check_outputs(o_gpu, o_ref, S, frac_flip=2e-3):
    err = np.abs(o_gpu - o_ref)
    tight = err <= 1e-5 * S
    assert np.all(err <= 2.0 ** -8 * S + 1e-5 * S), np.max(err / S)
    assert np.mean(~tight) <= frac_flip, np.mean(~tight)


@pytest.mark.parametrize("N", [1, 16, 1000, 40013])
def test_forward_parity(N):
    import paper_2109_00485_amd as L
    torch = torch_cuda()
    p = as_f32_params(params(1))
    rng = np.random.default_rng(N)
    f = features(rng, N).astype(np.float32)
    net = L.Mlp(blob(p))
    o = net.forward(to_dev(f, np.float32)).cpu().numpy().astype(np.float64)
    o_ref, S = scale_of(p, OM.standardize(p, f.astype(np.float64)))
    check_outputs(o, o_ref, S)
    torch.cuda.synchronize()


def test_forward_zero_output_and_empty():
    import paper_2109_00485_amd as L
    torch = torch_cuda()
    p = params(2)
    p.w3[:] = 0.0
    p.b3 = 0.0
    net = L.Mlp(blob(p))
    f = to_dev(features(np.random.default_rng(0), 333), np.float32)
    assert torch.all(net.forward(f) == 0)
    net.forward(f[:0])   # N = 0 is a no-op


@pytest.mark.parametrize("f32,offset", [(False, 0.0), (True, 0.0), (True, 1.5)])
@pytest.mark.parametrize("k", [1, 8, 13])
def test_precond_apply_parity(f32, k, offset):
    import paper_2109_00485_amd as L
    torch = torch_cuda()
    A = W.make_matrix("random_sym_1k")
    ctx = upload(A, f32)
    rho, tm = (x.cpu().numpy().astype(np.float64) for x in ctx.features())
    p = as_f32_params(params(3, mu=(100.0, 0.0, float(rho.mean()), float(tm.mean())),
                             sigma=(60.0, 20.0, float(rho.std()), float(tm.std() + 1e-3))))
    net = L.Mlp(blob(p))
    ctx.set_mlp(net)
    ctx.set_precond_offset(offset)
    rng = np.random.default_rng(k)
    dt = np.float32 if f32 else np.float64
    R = rng.standard_normal((A.n, k)).astype(dt)
    theta = np.sort(rng.uniform(-10, 10, k))
    theta[0] = float(np.asarray(A.diag, dtype=dt)[5])   # an exact shift: the guard applies
    Wg = ctx.precond_apply(to_dev(R, dt), to_dev(theta, np.float64), kind=L.PRECOND_MLP).cpu().numpy()
    d = np.asarray(A.diag, dtype=dt).astype(np.float64)
    eps = 1e-5 * ctx.query()["gamma"]
    m_ref = OM.precond_scale(p, d, theta, rho, tm, eps, a1_f32=True, offset=offset)
    W_ref = m_ref * R.astype(np.float64)
    # per-entry: the output error of the network plus the rounding of W
    f = np.empty((A.n, k, 4))
    f[:, :, 0] = d[:, None]
    f[:, :, 1] = theta[None, :]
    f[:, :, 2] = rho[:, None]
    f[:, :, 3] = tm[:, None]
    _, S = scale_of(p, OM.standardize(p, f.reshape(-1, 4)))
    S = S.reshape(A.n, k)
    rel = np.abs(Wg - W_ref) / np.maximum(np.abs(W_ref), 1e-300)
    ulp = 2.0 ** -23 if f32 else 2.0 ** -52
    tight = rel <= 1e-5 * S + 4 * ulp
    assert np.all(rel <= (2.0 ** -8 + 1e-5) * S + 4 * ulp)
    assert np.mean(~tight) <= 2e-3
    torch.cuda.synchronize()


def test_precond_apply_without_network_fails():
    import paper_2109_00485_amd as L
    torch = torch_cuda()
    A = W.make_matrix("random_sym_1k")
    ctx = upload(A, False)
    R = to_dev(np.ones((A.n, 2)), np.float64)
    th = to_dev(np.zeros(2), np.float64)
    with pytest.raises(L.LobpcgError) as e:
        ctx.precond_apply(R, th, kind=L.PRECOND_MLP)
    assert e.value.status == L.EINVAL
    torch.cuda.synchronize()


def make_batch(rng, ngroups, k, sizes=(1, 300)):
    cnt = rng.integers(sizes[0], sizes[1], ngroups)
    off = np.concatenate([[0], np.cumsum(cnt)]).astype(np.int64)
    N = int(off[-1])
    feat = features(rng, N).astype(np.float32)
    U = (rng.standard_normal(N) * 0.3).astype(np.float32)
    T = (U * rng.uniform(0.5, 1.5, N) + rng.standard_normal(N) * 0.05).astype(np.float32)
    w = rng.uniform(0.5, 20.0, N).astype(np.float32)
    X = (rng.standard_normal((N, k)) * 0.05).astype(np.float32)
    gid = np.repeat(np.arange(ngroups), cnt)
    return off, feat, U, T, w, X, gid


def device_batch(off, feat, U, T, w, X):
    import paper_2109_00485_amd as L
    return L.Batch(to_dev(feat, np.float32), to_dev(U, np.float32), to_dev(T, np.float32), to_dev(w, np.float32),
                   to_dev(X, np.float32), to_dev(off, np.int64))


def grad_blocks(g):
    return dict(W1=g[0:256], b1=g[256:320], W2=g[320:4416], b2=g[4416:4480], w3=g[4480:4544], b3=g[4544:4545])


def check_grad(g, g_ref):
    """Per parameter block: FP32 accumulation error, relative to the block's norm
    and, for a block whose exact gradient vanishes (b3: the loss does not see a
    common scale of the group's direction), to the whole gradient's norm."""
    gb = grad_blocks(g.astype(np.float64))
    total = np.sqrt(sum(np.sum(np.asarray(v, dtype=np.float64) ** 2) for v in g_ref.values()))
    for key, ref in g_ref.items():
        ref = np.asarray(ref, dtype=np.float64).ravel()
        err = np.linalg.norm(gb[key].ravel() - ref)
        assert err <= 1e-4 * np.linalg.norm(ref) + 1e-6 * total, (key, err, np.linalg.norm(ref))


@pytest.mark.parametrize("k", [3, 8])
def test_loss_and_gradient_parity(k):
    import paper_2109_00485_amd as L
    torch = torch_cuda()
    rng = np.random.default_rng(10 + k)
    off, feat, U, T, w, X, gid = make_batch(rng, 37, k)
    p = as_f32_params(params(4))
    net = L.Mlp(blob(p))
    loss, g = net.loss_grad(device_batch(off, feat, U, T, w, X))
    f64 = lambda a: np.asarray(a, dtype=np.float64)
    L_ref, g_ref = OM.group_loss(p, f64(feat), f64(U), f64(T), f64(w), f64(X), gid, 37, a1_f32=True)
    assert abs(loss - L_ref) <= 1e-6 * abs(L_ref) + 1e-9
    check_grad(g, g_ref)
    torch.cuda.synchronize()


def test_degenerate_and_empty_groups():
    import paper_2109_00485_amd as L
    torch = torch_cuda()
    rng = np.random.default_rng(5)
    off, feat, U, T, w, X, gid = make_batch(rng, 6, 4)
    T[gid == 2] = 0.0                                  # no target
    off = np.insert(off, 4, off[4])                    # an empty group (index 4)
    gid = np.repeat(np.arange(7), np.diff(off))
    p = as_f32_params(params(6))
    net = L.Mlp(blob(p))
    loss, g = net.loss_grad(device_batch(off, feat, U, T, w, X))
    f64 = lambda a: np.asarray(a, dtype=np.float64)
    L_ref, g_ref = OM.group_loss(p, f64(feat), f64(U), f64(T), f64(w), f64(X), gid, 7, a1_f32=True)
    assert abs(loss - L_ref) <= 1e-6 * abs(L_ref) + 1e-9
    check_grad(g, g_ref)
    # malformed offsets are rejected before any kernel indexes with them
    bad = off.copy()
    bad[3] = bad[2] - 1
    with pytest.raises(L.LobpcgError) as e:
        net.loss_grad(device_batch(bad, feat, U, T, w, X))
    assert e.value.status == L.EINVAL
    torch.cuda.synchronize()


def test_adam_step_parity():
    import paper_2109_00485_amd as L
    torch = torch_cuda()
    rng = np.random.default_rng(21)
    off, feat, U, T, w, X, gid = make_batch(rng, 20, 8)
    p = as_f32_params(params(7))
    net = L.Mlp(blob(p))
    lr = 1e-3
    f64 = lambda a: np.asarray(a, dtype=np.float64)
    st = OM.adam_init(p)
    q = p
    b = device_batch(off, feat, U, T, w, X)
    for step in range(3):
        loss = net.train_step(b, lr)
        L_ref, g_ref = OM.group_loss(q, f64(feat), f64(U), f64(T), f64(w), f64(X), gid, 20, a1_f32=True)
        # after the first step the FP32 Adam moments and weights have diverged from the
        # FP64 oracle's by rounding, which moves the loss at the 1e-6 level
        assert abs(loss - L_ref) <= (1e-6 if step == 0 else 1e-5) * abs(L_ref) + 1e-9
        q = as_f32_params(OM.adam_step(q, g_ref, st, lr))
        got = L.unpack_params(net.params())
        diffs = []
        for key in OM.Params.NAMES:
            ref = np.atleast_1d(np.asarray(getattr(q, key), dtype=np.float64))
            gk = np.atleast_1d(np.asarray(got[key], dtype=np.float64)).reshape(ref.shape)
            # an Adam step moves each weight by about lr whatever the gradient's size,
            # so a weight whose exact gradient is at rounding level (b3) may differ by lr
            assert np.max(np.abs(gk - ref)) <= 2 * lr * (step + 1), key
            diffs.append(np.abs(gk - ref).ravel())
        assert np.median(np.concatenate(diffs)) <= 1e-3 * lr
    torch.cuda.synchronize()


def test_fit_standardizer():
    import paper_2109_00485_amd as L
    torch = torch_cuda()
    f = features(np.random.default_rng(8), 50001).astype(np.float32)
    net = L.Mlp(blob(params(9)))
    net.fit_standardizer(to_dev(f, np.float32))
    got = L.unpack_params(net.params())
    f64 = f.astype(np.float64)
    np.testing.assert_allclose(got["mu"], f64.mean(0), rtol=1e-6)
    np.testing.assert_allclose(got["sigma"], f64.std(0), rtol=1e-6)
    torch.cuda.synchronize()


def harvest_inputs(A, nev=5, k=8, seed=0):
    import oracle
    Hs = oracle.SymMatrix.from_csr(A)
    rng = np.random.default_rng(seed)
    X, _ = np.linalg.qr(rng.standard_normal((A.n, k)))
    HX = Hs @ X
    theta = np.sort(rng.uniform(-5, 5, k))
    dense = Hs @ np.eye(A.n)
    xs = np.linalg.eigh(dense)[1][:, :nev]
    rho = Hs.row_offdiag_abs()
    cnt = Hs.row_offdiag_count()
    t = np.zeros(A.n)
    for b0 in range(0, A.n, 64):
        c = cnt[b0:b0 + 64].sum()
        t[b0:b0 + 64] = rho[b0:b0 + 64].sum() / c if c > 0 else 0.0
    return X, HX, theta, np.ascontiguousarray(xs), rho, t, Hs.gershgorin()


@pytest.mark.parametrize("offset", [0.0, 2.0])
def test_harvest_block_parity(offset):
    import paper_2109_00485_amd as L
    torch = torch_cuda()
    A = W.make_matrix("random_sym_1k")
    ctx = upload(A, False)
    ctx.set_precond_offset(offset)
    X, HX, theta, xs, rho, t, gamma = harvest_inputs(A)
    hb = L.HarvestBuffer(20000, 64, 8, to_dev(xs, np.float64), 5, rows=100, seed=11)
    hb.h.ngroups = 2                      # groups already held: the new ones are 2..6
    ctx.harvest_block(to_dev(X, np.float64), to_dev(HX, np.float64), to_dev(theta, np.float64), hb)
    assert hb.ngroups == 7 and not hb.full
    ref = OH.harvest_block(X, HX, theta, xs, A.diag, rho, t, 1e-5 * gamma, rows=100, nev=5, seed=11, group0=2,
                           offset=offset)
    off = hb.group_off.cpu().numpy()
    rows = hb.row.cpu().numpy()
    f32 = lambda a: np.asarray(a, dtype=np.float32)
    for j, r in enumerate(ref):
        b, e = off[2 + j], off[3 + j]
        got_rows = rows[b:e]
        order = np.argsort(got_rows)
        # the same FP64 decision on both sides; a draw within 1e-12 of p may go either way
        diff = np.setxor1d(got_rows, r["row"])
        close = np.abs(r["u_all"][diff] - r["p_all"][diff]) <= 1e-12
        assert np.all(close), diff
        common, ig, ir = np.intersect1d(got_rows[order], r["row"], return_indices=True)
        sel = order[ig]
        for name, got, exp in (("T", hb.T, r["E"]), ("U", hb.U, r["U"]), ("w", hb.w, r["w"])):
            g = got[b:e].cpu().numpy()[sel]
            np.testing.assert_allclose(g, f32(exp[ir]), rtol=2e-7, atol=1e-30, err_msg=name)
        fe = hb.feat[b:e].cpu().numpy()[sel]
        np.testing.assert_allclose(fe, f32(r["feat"][ir]), rtol=2e-7)
        np.testing.assert_allclose(hb.Xrow[b:e].cpu().numpy()[sel], f32(r["Xrow"][ir]), rtol=0)
    torch.cuda.synchronize()


def test_harvest_capacity_limits():
    import paper_2109_00485_amd as L
    torch = torch_cuda()
    A = W.make_matrix("random_sym_1k")
    ctx = upload(A, False)
    X, HX, theta, xs, rho, t, gamma = harvest_inputs(A)
    cap = 150                             # about 1.5 groups of ~100 rows
    hb = L.HarvestBuffer(cap + 1000, 64, 8, to_dev(xs, np.float64), 5, rows=100, seed=3)
    hb.h.capacity = cap
    args = (to_dev(X, np.float64), to_dev(HX, np.float64), to_dev(theta, np.float64))
    ctx.harvest_block(*args, hb)
    assert hb.full and 1 <= hb.ngroups < 5
    off = hb.group_off.cpu().numpy()
    assert hb.nsamples == off[hb.ngroups] <= cap
    # nothing written at or beyond the capacity
    assert torch.all(hb.U[cap:] == 0) and torch.all(hb.w[cap:] == 0) and torch.all(hb.Xrow[cap:] == 0)
    # a full buffer takes no more groups
    n_before = hb.ngroups
    ctx.harvest_block(*args, hb)
    assert hb.ngroups == n_before
    # too few group slots: nothing is added
    hb2 = L.HarvestBuffer(10000, 3, 8, to_dev(xs, np.float64), 5, rows=100, seed=3)
    ctx.harvest_block(*args, hb2)
    assert hb2.full and hb2.ngroups == 0 and hb2.nsamples == 0
    torch.cuda.synchronize()


def test_zero_network_solve_matches_diagonal():
    """exp(0) = 1: the network preconditioner with zero output takes the
    diagonal preconditioner's steps."""
    import paper_2109_00485_amd as L
    torch = torch_cuda()
    A = W.make_matrix("random_sym_1k")
    ctx = upload(A, False)
    p = params(12)
    p.w3[:] = 0.0
    p.b3 = 0.0
    net = L.Mlp(blob(p))
    ctx.set_mlp(net)
    X0 = W.initial_block(A.n, 8, seed=1)
    r_d = ctx.solve(to_dev(X0, np.float64), 5, precond=L.PRECOND_DIAG)
    r_m = ctx.solve(to_dev(X0, np.float64), 5, precond=L.PRECOND_MLP)
    assert r_d.status == 0 and r_m.status == 0
    # W = R (1/s) against W = R / s: last-bit differences, which the iteration count
    # (not the converged eigenvalues) is sensitive to
    assert abs(r_d.iters - r_m.iters) <= max(5, r_d.iters // 10)
    np.testing.assert_allclose(r_m.evals[:5], r_d.evals[:5], rtol=1e-10)
    torch.cuda.synchronize()


def test_solve_harvest_collects_groups():
    """A solve with a harvest attached appends nev groups every `every` iterations."""
    import paper_2109_00485_amd as L
    torch = torch_cuda()
    A = W.make_matrix("random_sym_1k")
    ctx = upload(A, False)
    X0 = W.initial_block(A.n, 8, seed=1)
    ref = ctx.solve(to_dev(X0, np.float64), 5, tol=1e-9)
    assert ref.status == 0
    Xs = to_dev(X0, np.float64)
    ctx.solve(Xs, 5, tol=1e-9)
    xs = Xs[:, :5].contiguous()
    hb = L.HarvestBuffer(400000, 4000, 8, xs, 5, every=3, rows=64, seed=5)
    r = ctx.solve(to_dev(X0, np.float64), 5, tol=1e-6, harvest=hb)
    assert r.status == 0
    assert hb.ngroups == 5 * (r.iters // 3)
    off = hb.group_off.cpu().numpy()[:hb.ngroups + 1]
    assert off[0] == 0 and np.all(np.diff(off) >= 0) and off[-1] == hb.nsamples
    w = hb.w[:hb.nsamples].cpu().numpy()
    assert np.all(w >= 1.0)
    torch.cuda.synchronize()
