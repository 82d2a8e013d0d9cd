"""Pins for the learned-preconditioner oracle (oracle.mlp): BF16 rounding
against torch's own conversion, the forward pass against an independent
torch.nn implementation, the zero-output special case (exactly the diagonal
preconditioner), central finite differences of the group loss, the loss's
invariances, and the closed form of a first Adam step."""
import numpy as np
import pytest
import torch

from oracle import mlp


def test_bf16_round_matches_torch():
    rng = np.random.default_rng(0)
    x = np.concatenate([rng.standard_normal(10000) * 10.0 ** rng.integers(-8, 8, 10000),
                        # exact ties between two BF16 neighbours, both parities
                        np.array([1.0 + 2 ** -8, 1.0 + 3 * 2 ** -8, -(1.0 + 2 ** -8), 3.0 + 2 ** -7]),
                        np.array([0.0, -0.0, 1.0, 65504.0])])
    ref = torch.from_numpy(x.astype(np.float32)).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(mlp.bf16_round(x), ref)


def test_forward_matches_torch_nn():
    p = mlp.init_params(3, mu=[100, -1, 30, 0.4], sigma=[50, 0.5, 5, 0.1])
    rng = np.random.default_rng(1)
    p.w3 = rng.standard_normal(64) * 0.1
    p.b1 = rng.standard_normal(64) * 0.1
    p.b2 = rng.standard_normal(64) * 0.1
    p.b3 = 0.3
    f = np.column_stack([rng.uniform(0, 200, 500), rng.uniform(-2, 0, 500), rng.uniform(20, 40, 500),
                         rng.uniform(0.3, 0.5, 500)])
    o, _ = mlp.forward(p, mlp.standardize(p, f))

    def bf(a):
        return torch.as_tensor(np.asarray(a, dtype=np.float32)).to(torch.bfloat16).to(torch.float64)
    l1, l2, l3 = torch.nn.Linear(4, 64).double(), torch.nn.Linear(64, 64).double(), torch.nn.Linear(64, 1).double()
    with torch.no_grad():
        l1.weight.copy_(bf(p.W1)); l1.bias.copy_(torch.from_numpy(p.b1))
        l2.weight.copy_(bf(p.W2)); l2.bias.copy_(torch.from_numpy(p.b2))
        l3.weight.copy_(bf(p.w3)[None, :]); l3.bias.fill_(p.b3)
        z = (torch.from_numpy(f) - torch.tensor([100, -1, 30, 0.4.__float__()], dtype=torch.float64)) / \
            torch.tensor([50, 0.5, 5, 0.1], dtype=torch.float64)
        h1 = torch.relu(l1(z)).to(torch.float32).to(torch.bfloat16).to(torch.float64)
        ref = l3(torch.relu(l2(h1)))[:, 0].numpy()
    np.testing.assert_allclose(o, ref, rtol=1e-12, atol=1e-12)


def test_zero_output_is_diagonal():
    p = mlp.init_params(0)
    d = np.linspace(0, 10, 50)
    theta = np.array([-1.0, 0.0, 2.5])
    m = mlp.precond_scale(p, d, theta, np.ones(50), np.ones(50), eps=0.1)
    assert np.array_equal(m, 1.0 / mlp.guard(d[:, None] - theta[None, :], 0.1))



def test_zero_output_is_offset_diagonal():
    """With the shift moved c spreads below theta (sigma = theta - c (max - min)),
    a zero network is exactly the shifted diagonal step: spread 3.5, c = 2 gives
    sigma = theta - 7."""
    p = mlp.init_params(0)
    d = np.linspace(0, 10, 50)
    theta = np.array([-1.0, 0.0, 2.5])
    m = mlp.precond_scale(p, d, theta, np.ones(50), np.ones(50), eps=0.1, offset=2.0)
    assert np.array_equal(m, 1.0 / mlp.guard(d[:, None] - (theta - 7.0)[None, :], 0.1))

def synthetic_batch(seed, ngroups=6, per=40, k=3):
    rng = np.random.default_rng(seed)
    N = ngroups * per
    gid = np.repeat(np.arange(ngroups), per)
    feat = np.column_stack([rng.uniform(0, 200, N), rng.uniform(-2, 0, N), rng.uniform(20, 40, N),
                            rng.uniform(0.3, 0.5, N)])
    X = rng.standard_normal((N, k)) * 0.1
    U = rng.standard_normal(N)
    T = rng.standard_normal(N)
    w = rng.uniform(0.5, 2.0, N)
    return feat, U, T, w, X, gid, ngroups


def test_group_loss_gradient_finite_differences():
    p = mlp.init_params(5, mu=[100, -1, 30, 0.4], sigma=[60, 0.6, 6, 0.06])
    rng = np.random.default_rng(2)
    p.w3 = rng.standard_normal(64) * 0.2
    p.b1 = rng.standard_normal(64) * 0.2
    p.b2 = rng.standard_normal(64) * 0.2
    batch = synthetic_batch(7)
    L, g = mlp.group_loss(p, *batch, bf16=False)
    h = 1e-6
    for name, idx in (("W1", (3, 1)), ("W1", (10, 3)), ("b1", (5,)), ("W2", (7, 20)), ("W2", (63, 0)),
                      ("b2", (11,)), ("w3", (9,)), ("w3", (40,)), ("b3", None)):
        def loss_at(delta):
            q = p.copy()
            if idx is None:
                q.b3 = p.b3 + delta
            else:
                arr = getattr(q, name)
                arr[idx] += delta
            return mlp.group_loss(q, *batch, with_grad=False, bf16=False)[0]
        fd = (loss_at(h) - loss_at(-h)) / (2 * h)
        an = g[name] if idx is None else g[name][idx]
        assert an == pytest.approx(fd, rel=1e-5, abs=1e-9), (name, idx, an, fd)


def test_group_loss_invariances():
    p = mlp.init_params(1)
    feat, U, T, w, X, gid, ng = synthetic_batch(3)
    L1, _ = mlp.group_loss(p, feat, U, T, w, X, gid, ng, with_grad=False)
    L2, _ = mlp.group_loss(p, feat, 7.5 * U, -3.0 * T, w, X, gid, ng, with_grad=False)
    assert L1 == pytest.approx(L2, rel=1e-12)
    assert 0.0 <= L1 <= 1.0
    # a direction equal to the target (with nothing in span(X)) has zero loss
    X0 = np.zeros_like(X)
    L0, _ = mlp.group_loss(p, feat, T.copy(), T, w, X0, gid, ng, with_grad=False)
    assert abs(L0) < 1e-14


def test_first_adam_step_closed_form():
    p = mlp.init_params(2)
    g = {k: np.asarray(getattr(p, k), dtype=np.float64) * 0 + 0.3 for k in mlp.Params.NAMES}
    g["W1"] = np.full_like(p.W1, -2.0)
    st = mlp.adam_init(p)
    q = mlp.adam_step(p, g, st, lr=1e-2)
    # bias-corrected first step moves every weight by -lr * g / (|g| + eps)
    np.testing.assert_allclose(q.W1 - p.W1, 1e-2 * 2.0 / (2.0 + 1e-8), rtol=1e-12)
    np.testing.assert_allclose(q.W2 - p.W2, -1e-2 * 0.3 / (0.3 + 1e-8), rtol=1e-12)


def test_degenerate_group_has_zero_loss_and_gradient():
    p = mlp.init_params(0)
    rng = np.random.default_rng(2)
    p.w3 = rng.standard_normal(64) * 0.1
    n, k = 60, 4
    feat = rng.standard_normal((n, 4))
    U, T, w = rng.standard_normal(n), rng.standard_normal(n), rng.uniform(0.5, 2, n)
    X = rng.standard_normal((n, k)) * 0.1
    gid = np.repeat([0, 1], n // 2)
    T0 = T.copy()
    T0[gid == 1] = 0.0   # group 1 has no target
    L, g = mlp.group_loss(p, feat, U, T0, w, X, gid, 2)
    L_a, g_a = mlp.group_loss(p, feat[gid == 0], U[gid == 0], T0[gid == 0], w[gid == 0], X[gid == 0],
                              np.zeros(n // 2, dtype=int), 1)
    # group 1 contributes 0 to the mean over two groups and nothing to the gradient
    assert np.isclose(L, L_a / 2, rtol=1e-13)
    for key in g:
        assert np.allclose(np.asarray(g[key]) * 2, np.asarray(g_a[key]), rtol=1e-12, atol=1e-15)


def test_fp32_first_layer_exact_on_representable_inputs():
    """With inputs on a coarse grid every FP32 first-layer sum is exact, so the
    FP32 decision path and the FP64 path coincide bit for bit."""
    p = mlp.init_params(5)
    rng = np.random.default_rng(3)
    p.W1 = mlp.bf16_round(p.W1)
    p.b1 = np.round(rng.standard_normal(64) * 8) / 8
    p.w3 = rng.standard_normal(64) * 0.1
    z = np.round(rng.standard_normal((300, 4)) * 4) / 4
    o64, _ = mlp.forward(p, z)
    o32, _ = mlp.forward(p, z, a1_f32=True)
    assert np.array_equal(o64, o32)


def test_bounded_scale():
    """exp(b(o)) with b = 2 tanh(o / 2): the learned factor on the diagonal step
    stays in [e^-2, e^2] however large the network output."""
    p = mlp.init_params(1)
    rng = np.random.default_rng(4)
    p.w3 = rng.standard_normal(64) * 50.0
    p.b3 = 3.0
    n, k = 500, 3
    d = rng.uniform(0, 100, n)
    theta = np.array([-1.0, 20.0, 50.0])
    rho, tm = rng.uniform(10, 20, n), rng.uniform(0.2, 0.4, n)
    m = mlp.precond_scale(p, d, theta, rho, tm, eps=1e-3)
    base = 1.0 / mlp.guard(d[:, None] - theta[None, :], 1e-3)
    r = m / base
    assert np.all(r >= np.exp(-2.0) * (1 - 1e-12)) and np.all(r <= np.exp(2.0) * (1 + 1e-12))
    assert r.max() > 5.0 and r.min() < 0.2        # the bound is actually reached here
    assert np.allclose(mlp.bound([0.0, 1e9, -1e9]), [0.0, 2.0, -2.0])


def test_group_loss_hand_computed_with_span_x():
    """Two groups of three rows, k = 1, X != 0, and a zero output layer (so the
    learned factor is exp(0) = 1 and u = U).  Worked by hand from the loss's
    definition:
      group 0: w = (2, 1, 1), x = (1, 0, 1), U = (1, 2, 3), T = (1, 1, -1)
               a = sum w x u = 2 + 0 + 3 = 5,  u' = u - x a = (-4, 2, -2)
               sum w u' T = -8 + 2 + 2 = -4,  sum w u'^2 = 32 + 4 + 4 = 40,
               sum w T^2 = 4,  L_0 = 1 - 16 / 160 = 9/10
      group 1: w = (1/2, 1, 2), x = (2, -1, 0), U = (1, 0, 1), T = (0, 2, 1)
               a = 1 + 0 + 0 = 1,  u' = (-1, 1, 1)
               sum w u' T = 0 + 2 + 2 = 4,  sum w u'^2 = 1/2 + 1 + 2 = 7/2,
               sum w T^2 = 0 + 4 + 2 = 6,  L_1 = 1 - 16 / 21 = 5/21
      loss = (9/10 + 5/21) / 2 = 239/420.
    A projection coefficient without the weights (a_0 = 4) or summed over both
    groups (a = 6) gives another value."""
    p = mlp.init_params(0)            # w3 = 0, b3 = 0: zero output
    feat = np.zeros((6, 4))
    U = np.array([1.0, 2.0, 3.0, 1.0, 0.0, 1.0])
    T = np.array([1.0, 1.0, -1.0, 0.0, 2.0, 1.0])
    w = np.array([2.0, 1.0, 1.0, 0.5, 1.0, 2.0])
    X = np.array([[1.0], [0.0], [1.0], [2.0], [-1.0], [0.0]])
    gid = np.array([0, 0, 0, 1, 1, 1])
    L, _ = mlp.group_loss(p, feat, U, T, w, X, gid, 2, with_grad=False)
    assert L == pytest.approx(239.0 / 420.0, rel=1e-14)
    # each group alone
    L0, _ = mlp.group_loss(p, feat[:3], U[:3], T[:3], w[:3], X[:3], np.zeros(3, dtype=int), 1, with_grad=False)
    L1, _ = mlp.group_loss(p, feat[3:], U[3:], T[3:], w[3:], X[3:], np.zeros(3, dtype=int), 1, with_grad=False)
    assert L0 == pytest.approx(0.9, rel=1e-14) and L1 == pytest.approx(5.0 / 21.0, rel=1e-14)


def test_group_loss_target_in_span_x_is_orthogonal():
    """With X orthonormal in the group's weighted inner product (X^T diag(w) X = I),
    the projected direction u' = u - X (X^T diag(w) u) is w-orthogonal to span(X);
    a target T inside span(X) therefore has cosine 0 with u' and the group's loss
    is exactly 1, whatever u.  A projection without the weights leaves a component
    along T."""
    rng = np.random.default_rng(11)
    N, k = 40, 3
    w = rng.uniform(0.5, 2.0, N)
    A = rng.standard_normal((N, k))
    # weighted Gram-Schmidt via the Cholesky factor of A^T W A
    Lc = np.linalg.cholesky(A.T @ (w[:, None] * A))
    X = np.linalg.solve(Lc, A.T).T
    assert np.allclose(X.T @ (w[:, None] * X), np.eye(k), atol=1e-12)
    T = X @ np.array([0.7, -1.3, 0.4])
    p = mlp.init_params(2)
    p.w3 = rng.standard_normal(64) * 0.3   # a non-trivial learned factor
    feat = rng.standard_normal((N, 4))
    U = rng.standard_normal(N)
    L, _ = mlp.group_loss(p, feat, U, T, w, X, np.zeros(N, dtype=int), 1, with_grad=False)
    assert L == pytest.approx(1.0, abs=1e-12)


def test_adam_three_steps_match_torch():
    """Three Adam steps with different gradients each step against torch.optim.Adam
    (an independent implementation of Kingma & Ba's update with bias corrections
    1 - beta^t): the bias correction's power of t shows from the second step on,
    which a first step alone cannot reveal."""
    import torch
    p = mlp.init_params(4)
    rng = np.random.default_rng(5)
    grads = []
    for t in range(3):
        g = {k: rng.standard_normal(np.shape(getattr(p, k))) * (1.0 + t) for k in mlp.Params.NAMES}
        g["b3"] = float(rng.standard_normal())
        grads.append(g)
    lr = 3e-3
    st = mlp.adam_init(p)
    q = p
    tens = {k: torch.tensor(np.asarray(getattr(p, k), dtype=np.float64), requires_grad=True)
            for k in mlp.Params.NAMES}
    opt = torch.optim.Adam(list(tens.values()), lr=lr, betas=(0.9, 0.999), eps=1e-8)
    for g in grads:
        q = mlp.adam_step(q, g, st, lr=lr)
        opt.zero_grad()
        for k, tt in tens.items():
            tt.grad = torch.tensor(np.asarray(g[k], dtype=np.float64))
        opt.step()
        for k, tt in tens.items():
            np.testing.assert_allclose(np.asarray(getattr(q, k), dtype=np.float64), tt.detach().numpy(),
                                       rtol=1e-13, atol=1e-15)
    assert st.t == 3
