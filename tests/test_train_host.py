"""Host-side logic of the training driver: the BF16 rounding used by sample
shards agrees with torch's float32 -> bfloat16 conversion (round to nearest
even), and a shard file keeps the group offsets and the FP32 features."""
import json

import numpy as np


def test_bf16_rounding_matches_torch():
    import torch
    from paper_2109_00485_amd.train import _bf16_bits, _bf16_value
    rng = np.random.default_rng(0)
    x = np.concatenate([rng.standard_normal(10000) * 10.0 ** rng.integers(-30, 30, 10000),
                        [0.0, -0.0, 1.0, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -8, 65504.0, 1e-40]]).astype(np.float32)
    ours = _bf16_value(_bf16_bits(x))
    ref = torch.from_numpy(x).to(torch.bfloat16).to(torch.float32).numpy()
    assert np.array_equal(ours.view(np.uint32), ref.view(np.uint32))


def test_shard_file_layout(tmp_path):
    import torch
    from paper_2109_00485_amd.train import _bf16_value, save_shard

    class B:
        pass
    b = B()
    n, k = 50, 8
    rng = np.random.default_rng(1)
    feat = torch.from_numpy(rng.standard_normal((n, 4)).astype(np.float32))
    vec = [torch.from_numpy(rng.standard_normal(n).astype(np.float32)) for _ in range(3)]
    X = torch.from_numpy(rng.standard_normal((n, k)).astype(np.float32))
    goff = torch.tensor([0, 20, 35, 50], dtype=torch.int64)
    b.t = (feat, *vec, X, goff)
    p = tmp_path / "s.npz"
    save_shard(str(p), b, {"train_seeds": "0:2", "runs": [{"seed": 0}]})
    with np.load(p, allow_pickle=False) as z:
        assert np.array_equal(z["feat"], feat.numpy())
        assert np.array_equal(z["group_off"], goff.numpy())
        assert z["Xrow"].shape == (n, k)
        assert np.allclose(_bf16_value(z["U"]), vec[0].numpy(), rtol=2 ** -8)
        assert json.loads(bytes(z["meta"]).decode())["train_seeds"] == "0:2"
