"""The learned preconditioner end to end on the GPU: harvest training samples
from plain diagonal-preconditioned solves (exact corrections from a tight FP64
pass of the same matrix), fit the network with the library's training
kernels, and solve held-out matrices with the diagonal and with the trained
network.  What the network gains has no reference (parity unpinned): the test
asserts that it converges to the same eigenvalues in fewer iterations."""
import numpy as np
import pytest
import torch

from synth import workloads as W

pytestmark = pytest.mark.gpu


def test_trained_network_beats_diagonal():
    import paper_2109_00485_amd as L
    from paper_2109_00485_amd import train
    assert torch.cuda.is_available()
    n = 20000
    dummy = torch.zeros((1, 5), dtype=torch.float64, device="cuda")
    hb = L.HarvestBuffer(2_000_000, 20_000, 8, dummy, 5, every=3, rows=256)
    for seed in range(4):
        A = W.make_matrix("random_sym_20k", seed=seed, n=n, f32=False)
        info = train.harvest_matrix(A, hb, every=3, rows=256, seed=seed)
        assert info["status"] == 0 and info["star_status"] == 0
    assert hb.ngroups > 1000 and not hb.full
    batch = hb.batch()
    net = L.Mlp(train.init_params(0))
    net.fit_standardizer(batch.t[0])
    losses = train.fit(net, batch, steps=400, log_every=0)
    assert losses[-1] < losses[0]
    gains = []
    for seed in (1000, 1001):
        A = W.make_matrix("random_sym_20k", seed=seed, n=n, f32=True)
        r = train.compare(A, net)
        assert r["diag"]["status"] == 0 and r["mlp"]["status"] == 0
        ed, em = np.array(r["diag"]["evals"]), np.array(r["mlp"]["evals"])
        # both runs pass their own 1e-6 residual test; their values agree far inside 1e-5
        assert np.all(np.abs(ed - em) <= 1e-5 * np.maximum(np.abs(ed), 1.0)), (ed, em)
        gains.append(r["diag"]["iters"] / r["mlp"]["iters"])
        print(f"seed {seed}: diag {r['diag']['iters']} it, mlp {r['mlp']['iters']} it")
    assert min(gains) > 1.25, gains
