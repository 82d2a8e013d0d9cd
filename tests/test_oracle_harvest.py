"""Pins for the training-sample harvest oracle (oracle.harvest): the SplitMix64
generator against its published output sequence, the correction's
orthogonality to span(X), the inclusion probabilities' closed forms, and the
unbiasedness of the importance-weighted sums (Horvitz-Thompson)."""
import numpy as np

from oracle import harvest as H


def test_splitmix64_published_sequence():
    import os
    path = os.path.join(os.path.dirname(__file__), "golden", "splitmix64_seed1234567.txt")
    ref = [int(l) for l in open(path) if l.strip() and not l.startswith("#")]
    assert len(ref) == 5
    assert [int(x) for x in H.splitmix64_sequence(1234567, 5)] == ref


def test_uniform_range_and_moments():
    u = H.uniform(7, 3, np.arange(200000))
    assert u.min() >= 0.0 and u.max() < 1.0
    assert abs(u.mean() - 0.5) < 3e-3 and abs(u.var() - 1 / 12) < 2e-3
    # distinct groups give different streams
    assert not np.array_equal(u[:100], H.uniform(7, 4, np.arange(100)))


def _setup(n=400, k=8, nev=5, seed=0):
    rng = np.random.default_rng(seed)
    X, _ = np.linalg.qr(rng.standard_normal((n, k)))
    xs, _ = np.linalg.qr(rng.standard_normal((n, nev)))
    A = rng.standard_normal((n, n)) * 0.1
    Hm = np.diag(np.sort(rng.uniform(0, 10, n))) + (A + A.T)
    return rng, X, Hm @ X, rng.uniform(-1, 1, k), xs, np.diag(Hm)


def test_correction_orthogonal_to_block():
    rng, X, HX, th, xs, d = _setup()
    out = H.harvest_block(X, HX, th, xs, d, np.ones(400), np.ones(400), 1e-3, rows=800, nev=5, seed=1, group0=0)
    for j, g in enumerate(out):
        E = np.zeros(400)
        E[g["row"]] = g["E"]
        # rows = 2n keeps every row (p = 1): the full correction, orthogonal to X
        assert g["row"].size == 400 and np.allclose(g["w"], 1.0)
        assert np.abs(X.T @ E).max() < 1e-12
        # E + X X^T x* = x*
        assert np.allclose(E + X @ (X.T @ xs[:, j]), xs[:, j], atol=1e-14)


def test_probabilities_closed_forms():
    rng, X, HX, th, xs, d = _setup()
    out = H.harvest_block(X, HX, th, xs, d, np.ones(400), np.ones(400), 1e-3, rows=16, nev=5, seed=1, group0=0)
    for g in out:
        # no clipping at rows=16: the probabilities sum to rows exactly
        assert g["p_all"].max() < 1.0
        assert abs(g["p_all"].sum() - 16.0) < 1e-10
        # kept exactly where the draw is below the probability
        assert np.array_equal(np.nonzero(g["u_all"] < g["p_all"])[0], g["row"])
    # x* = 0: E = 0 and the draw is uniform with p = rows / n
    out = H.harvest_block(X, HX, th, np.zeros((400, 5)), d, np.ones(400), np.ones(400), 1e-3, rows=16, nev=5,
                          seed=1, group0=0)
    for g in out:
        assert np.allclose(g["p_all"], 16 / 400)


def test_weighted_sums_unbiased():
    rng, X, HX, th, xs, d = _setup(n=300)
    f = rng.standard_normal(300)
    est = []
    for seed in range(3000):
        g = H.harvest_block(X, HX, th, xs, d, np.ones(300), np.ones(300), 1e-3, rows=20, nev=1, seed=seed,
                            group0=5)[0]
        est.append(np.sum(g["w"] * f[g["row"]]))
    est = np.array(est)
    # Horvitz-Thompson: E[sum w f] = sum f; 5-sigma band of the Monte Carlo mean
    assert abs(est.mean() - f.sum()) < 5 * est.std() / np.sqrt(est.size)


def test_residual_step_fields():
    rng, X, HX, th, xs, d = _setup()
    eps = 1e-3
    th[0] = d[7]  # exact shift: the guard applies at row 7
    out = H.harvest_block(X, HX, th, xs, d, np.arange(400.0), np.arange(400.0) * 2, eps, rows=800, nev=1,
                          seed=0, group0=0)[0]
    R = HX[:, 0] - X[:, 0] * th[0]
    den = d - th[0]
    assert out["U"][7] == R[7] / eps
    mask = np.abs(den) >= eps
    assert np.allclose(out["U"][mask] * den[mask], R[mask], rtol=1e-14, atol=1e-15)
    assert np.array_equal(out["feat"][:, 2], np.arange(400.0)) and np.all(out["feat"][:, 1] == th[0])



def test_residual_step_with_shift_offset():
    """U_ij = R_ij / s(d_i - sigma_j), sigma_j = theta_j - c (max theta - min theta):
    the harvested step is the shifted diagonal step (here computed by hand)."""
    rng, X, HX, th, xs, d = _setup()
    eps = 1e-3
    c = 3.0
    out = H.harvest_block(X, HX, th, xs, d, np.arange(400.0), np.arange(400.0) * 2, eps, rows=800, nev=2,
                          seed=0, group0=0, offset=c)
    for j in range(2):
        R = HX[:, j] - X[:, j] * th[j]
        sigma = th[j] - c * (th.max() - th.min())
        den = d - sigma
        o = out[j]
        mask = np.abs(den[o["row"]]) >= eps
        assert np.allclose(o["U"][mask] * den[o["row"]][mask], R[o["row"]][mask], rtol=1e-14, atol=1e-15)
        assert np.all(o["feat"][:, 1] == th[j])      # the feature stays the Ritz value itself
