"""Helpers for the GPU parity tests (inputs from synth, expectations from oracle)."""
from __future__ import annotations

import numpy as np


def torch_cuda():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    return torch


def upload(A, f32: bool, fmt=None, **kw):
    """Context for the upper-triangle CSR ``A`` (values cast to the context dtype)."""
    import paper_2109_00485_amd as L
    torch = torch_cuda()
    val = np.asarray(A.val, dtype=np.float32 if f32 else np.float64)

    class _A:
        pass
    a = _A()
    a.n, a.row_ptr, a.col, a.val = A.n, A.row_ptr, A.col, val
    return L.Context.from_csr(a, dtype=L.F32 if f32 else L.F64, fmt=L.FORMAT_AUTO if fmt is None else fmt, **kw)


def to_dev(x, dtype):
    torch = torch_cuda()
    return torch.from_numpy(np.ascontiguousarray(x, dtype=dtype)).cuda()


def row_error(Y, Yref, Yabs):
    """max_i ||Y_i - Yref_i|| / ||(|H||X|)_i||  (rows with zero scale must match exactly)."""
    num = np.linalg.norm(np.asarray(Y, dtype=np.float64) - Yref, axis=1)
    den = np.linalg.norm(Yabs, axis=1)
    zero = den == 0
    assert np.all(num[zero] == 0)
    return float(np.max(num[~zero] / den[~zero])) if np.any(~zero) else 0.0
