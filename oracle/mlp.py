"""FP64 oracle of the learned preconditioner network (test infrastructure).

The network replaces the diagonal shift-inverse 1/s(d_i - sigma_j) of the
preconditioner (Section 3.4 with 1 x 1 tiles; sigma_j = theta_j unless an
offset moves the shift, see oracle.precond) by a learned per-entry scale

    m_ij = exp(b(o_ij)) / s(d_i - sigma_j),   W_ij = m_ij R_ij,
    b(o) = C tanh(o / C),  C = OUT_BOUND = 2,

so the network can reweight an entry of the diagonal step by a factor in
[e^-2, e^2] but never suppress or blow up a row (an unbounded exp(o) let
trained networks zero out most rows and stall the iteration),

where o_ij = f(z_ij) is a 4 -> 64 -> 64 -> 1 MLP of the standardised inputs
z = (f - mu) / sigma, f = (d_i, theta_j, rho_i, t_i): the diagonal entry, the
Ritz value, the full-row off-diagonal 1-norm sum_{j != i} |h_ij|, and the mean
|h| over the off-diagonal nonzeros of the 64-row tile containing row i.
A network whose output is zero reproduces the diagonal preconditioner exactly.

Precision (shared with the GPU kernels): W1, W2, w3 are held in FP32 and used
rounded to BF16 (round to nearest even); the first hidden activation is
rounded to BF16 before the second layer (the matrix-core operand); biases,
accumulations and everything else are FP32 on the GPU and FP64 here.

Training loss, per group g = (run, iteration, column j) of harvested rows i
with importance weights w_i (the rows are a sample of the column):
    u_i  = exp(b(o_i)) U_i              U = R / s(d - theta): the diagonal step
    u'_i = u_i - x_i^T a,  a = sum_l w_l x_l u_l    (remove the span(X) part)
    L_g  = 1 - (sum w u' T)^2 / ((sum w u'^2)(sum w T^2))
with T the exact correction of the column (its error outside span(X)).  L_g is
invariant to the scale of the direction, which the Rayleigh-Ritz step does not
see either; the loss is the mean over groups.  A group with sum w u'^2 = 0 or
sum w T^2 = 0 has no defined angle and contributes 0 with zero gradient.  Parity of what the trained
network gains is unpinned: it is measured by iteration counts, not by a
reference.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

NIN, HID = 4, 64
OUT_BOUND = 2.0


def bound(o):
    """b(o) = C tanh(o / C): the log-scale the preconditioner applies."""
    return OUT_BOUND * np.tanh(np.asarray(o, dtype=np.float64) / OUT_BOUND)


def bf16_round(x) -> np.ndarray:
    """Round to the nearest BF16 (ties to even) through the FP32 bit pattern."""
    x32 = np.ascontiguousarray(x, dtype=np.float32)
    b = x32.view(np.uint32).astype(np.uint64)
    b = (b + 0x7FFF + ((b >> 16) & 1)) & 0xFFFF0000
    return b.astype(np.uint32).view(np.float32).astype(np.float64).reshape(np.shape(x))


@dataclass
class Params:
    W1: np.ndarray   # HID x NIN
    b1: np.ndarray   # HID
    W2: np.ndarray   # HID x HID
    b2: np.ndarray   # HID
    w3: np.ndarray   # HID
    b3: float
    mu: np.ndarray   # NIN
    sigma: np.ndarray  # NIN

    NAMES = ("W1", "b1", "W2", "b2", "w3", "b3")

    def copy(self):
        return Params(**{k: np.array(getattr(self, k), dtype=np.float64) for k in
                         ("W1", "b1", "W2", "b2", "w3", "mu", "sigma")}, b3=float(self.b3))


def init_params(seed: int, mu=None, sigma=None) -> Params:
    """He-normal hidden layers, zero output layer (starts as the diagonal preconditioner)."""
    rng = np.random.default_rng(seed)
    W1 = rng.standard_normal((HID, NIN)) * np.sqrt(2.0 / NIN)
    W2 = rng.standard_normal((HID, HID)) * np.sqrt(2.0 / HID)
    return Params(W1=W1.astype(np.float32).astype(np.float64), b1=np.zeros(HID),
                  W2=W2.astype(np.float32).astype(np.float64), b2=np.zeros(HID), w3=np.zeros(HID), b3=0.0,
                  mu=np.zeros(NIN) if mu is None else np.asarray(mu, dtype=np.float64),
                  sigma=np.ones(NIN) if sigma is None else np.asarray(sigma, dtype=np.float64))


def standardize(p: Params, f: np.ndarray) -> np.ndarray:
    return (np.asarray(f, dtype=np.float64) - p.mu) / p.sigma


def forward(p: Params, z: np.ndarray, bf16: bool = True, a1_f32: bool = False):
    """o = w3 . relu(W2 bf16(relu(W1 z + b1)) + b2) + b3 with BF16 weights
    (``bf16=False`` evaluates the same network without the roundings).

    ``a1_f32``: form the first layer's pre-activations in FP32 (inputs, weights
    and sum rounded to FP32), the precision in which the kernels take the BF16
    rounding decision of the hidden activations; everything else stays FP64."""
    rnd = bf16_round if bf16 else (lambda a: np.asarray(a, dtype=np.float64))
    W1, W2, w3 = rnd(p.W1), rnd(p.W2), rnd(p.w3)
    if a1_f32:
        z32 = np.asarray(z, dtype=np.float32)
        a1 = (z32 @ W1.T.astype(np.float32) + np.asarray(p.b1, dtype=np.float32)).astype(np.float64)
    else:
        a1 = z @ W1.T + p.b1
    h1 = np.maximum(a1, 0.0)
    h1b = rnd(h1)
    a2 = h1b @ W2.T + p.b2
    h2 = np.maximum(a2, 0.0)
    o = h2 @ w3 + p.b3
    return o, (z, a1, h1b, a2, h2, W1, W2, w3)


def guard(x, eps):
    x = np.asarray(x, dtype=np.float64)
    return np.where(np.abs(x) >= eps, x, np.where(x < 0, -eps, eps))


def precond_scale(p: Params, d, theta, rownorm, tilemean, eps, a1_f32: bool = False,
                  offset: float = 0.0) -> np.ndarray:
    """m_ij (n x k) for every row i and Ritz value theta_j; non-finite -> diagonal.
    The diagonal step divides by s(d_i - sigma_j), sigma_j = theta_j - offset *
    (max theta - min theta) (offset 0: the Ritz value itself)."""
    d = np.asarray(d, dtype=np.float64)
    theta = np.asarray(theta, dtype=np.float64)
    n, k = d.size, theta.size
    f = np.empty((n, k, NIN))
    f[:, :, 0] = d[:, None]
    f[:, :, 1] = theta[None, :]
    f[:, :, 2] = np.asarray(rownorm, dtype=np.float64)[:, None]
    f[:, :, 3] = np.asarray(tilemean, dtype=np.float64)[:, None]
    o, _ = forward(p, standardize(p, f.reshape(-1, NIN)), a1_f32=a1_f32)
    o = o.reshape(n, k)
    sigma = theta - offset * (theta.max() - theta.min())
    base = 1.0 / guard(d[:, None] - sigma[None, :], eps)
    m = np.exp(bound(o)) * base
    return np.where(np.isfinite(m), m, base)


def group_loss(p: Params, feat, U, T, w, X, gid, ngroups, with_grad=True, bf16=True, a1_f32=False):
    """Mean group loss and (optionally) the gradients w.r.t. W1, b1, W2, b2, w3, b3.

    feat: N x 4 raw features; U, T, w: N; X: N x k (row i of the block X); gid: N ints.
    """
    z = standardize(p, feat)
    o, (z, a1, h1b, a2, h2, W1b, W2b, w3b) = forward(p, z, bf16=bf16, a1_f32=a1_f32)
    ob = bound(o)
    e = np.exp(ob)
    u = e * U
    k = X.shape[1]
    a = np.zeros((ngroups, k))
    np.add.at(a, gid, (w * u)[:, None] * X)
    up = u - np.einsum("ij,ij->i", X, a[gid])
    S_uT = np.bincount(gid, w * up * T, ngroups)
    S_uu = np.bincount(gid, w * up * up, ngroups)
    S_TT = np.bincount(gid, w * T * T, ngroups)
    # a group whose direction or target vanishes has no defined angle: loss 0, no gradient
    valid = (S_uu > 0) & (S_TT > 0)
    den = np.where(valid, S_uu * S_TT, 1.0)
    Lg = np.where(valid, 1.0 - S_uT ** 2 / den, 0.0)
    L = float(Lg.mean())
    if not with_grad:
        return L, None
    # dL/du'_i for the mean over groups
    coef = 1.0 / ngroups
    den2 = np.where(valid, S_uu ** 2 * S_TT, 1.0)
    g_up = np.where(valid[gid], -2.0 * w * (S_uT[gid] * T * S_uu[gid] - S_uT[gid] ** 2 * up) / den2[gid] * coef, 0.0)
    Gx = np.zeros((ngroups, k))
    np.add.at(Gx, gid, g_up[:, None] * X)
    g_u = g_up - w * np.einsum("ij,ij->i", X, Gx[gid])
    g_o = g_u * U * e * (1.0 - (ob / OUT_BOUND) ** 2)   # d b / d o = 1 - tanh^2
    # back through the network (straight-through for the BF16 roundings)
    g_w3 = h2.T @ g_o
    g_b3 = float(g_o.sum())
    g_h2 = np.outer(g_o, w3b)
    g_a2 = g_h2 * (a2 > 0)
    g_W2 = g_a2.T @ h1b
    g_b2 = g_a2.sum(0)
    g_h1 = g_a2 @ W2b
    g_a1 = g_h1 * (a1 > 0)
    g_W1 = g_a1.T @ z
    g_b1 = g_a1.sum(0)
    return L, dict(W1=g_W1, b1=g_b1, W2=g_W2, b2=g_b2, w3=g_w3, b3=g_b3)


@dataclass
class AdamState:
    m: dict
    v: dict
    t: int = 0


def adam_init(p: Params) -> AdamState:
    z = {k: np.zeros_like(np.asarray(getattr(p, k), dtype=np.float64)) for k in Params.NAMES}
    return AdamState(m=z, v={k: np.zeros_like(x) for k, x in z.items()})


def adam_step(p: Params, g: dict, st: AdamState, lr: float, b1=0.9, b2=0.999, eps=1e-8) -> Params:
    """One Adam step (Kingma & Ba, 2015) on the FP32 master weights."""
    st.t += 1
    q = p.copy()
    for k in Params.NAMES:
        gk = np.asarray(g[k], dtype=np.float64)
        st.m[k] = b1 * st.m[k] + (1 - b1) * gk
        st.v[k] = b2 * st.v[k] + (1 - b2) * gk * gk
        mh = st.m[k] / (1 - b1 ** st.t)
        vh = st.v[k] / (1 - b2 ** st.t)
        new = np.asarray(getattr(q, k), dtype=np.float64) - lr * mh / (np.sqrt(vh) + eps)
        setattr(q, k, float(new) if k == "b3" else new)
    return q
