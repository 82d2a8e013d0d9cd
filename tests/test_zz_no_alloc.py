"""The allocation-free Gram entry point (lobpcg_gram_noalloc, C ABI) against
the context entry point lobpcg_gram on the same inputs: bitwise on
integer-valued blocks (every summation order is exact there), within the Gram
parity bars otherwise, on consecutive calls with shrinking inputs (the static
scratch keeps the previous call's contents)."""
import ctypes

import numpy as np
import pytest

import synth
from gpu_util import to_dev, torch_cuda, upload

pytestmark = pytest.mark.gpu


def noalloc(a, b, prec, f32=True):
    import paper_2109_00485_amd as L
    torch = torch_cuda()
    lib = L.load()
    n, ka = a.shape
    kb = b.shape[1]
    G = torch.full((ka, kb), np.nan, dtype=torch.float64, device="cuda")
    rc = lib.lobpcg_gram_noalloc(ctypes.c_void_p(a.data_ptr()), ka, ctypes.c_void_p(b.data_ptr()), kb, n,
                                 L.F32 if f32 else L.F64, ctypes.c_void_p(G.data_ptr()), prec,
                                 ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert rc == L.OK, rc
    torch.cuda.synchronize()
    return G.cpu().numpy()


def test_noalloc_gram_matches_context_gram():
    import paper_2109_00485_amd as L
    torch = torch_cuda()
    rng = np.random.default_rng(11)
    # 1) large integer-valued FP32 blocks (more slabs than the scratch has workgroups): bitwise
    n1 = 200_003
    A1 = synth.random_sym(n1, 1, seed=2)
    c1 = upload(A1, True)
    a = rng.integers(-16, 17, size=(n1, 24)).astype(np.float32)
    b = rng.integers(-16, 17, size=(n1, 48)).astype(np.float32)
    da, db = to_dev(a, np.float32), to_dev(b, np.float32)
    ref = a.astype(np.float64).T @ b.astype(np.float64)
    for prec in (L.GRAM_F64, L.GRAM_F32, L.GRAM_BF16X3):
        Gn = noalloc(da, db, prec)
        Gc = c1.gram(da, db, prec=prec).cpu().numpy()
        assert np.array_equal(Gn, Gc) and np.array_equal(Gn, ref), prec
    c1.close()
    # 2) a smaller Gaussian FP32 call right after: within the FP32 / FP64 Gram bars
    n2 = 5003
    A2 = synth.random_sym(n2, 2, seed=1)
    c2 = upload(A2, True)
    a = synth.gaussian_block(n2, 8, seed=2).astype(np.float32)
    b = synth.gaussian_block(n2, 13, seed=3).astype(np.float32)
    da, db = to_dev(a, np.float32), to_dev(b, np.float32)
    ref = a.astype(np.float64).T @ b.astype(np.float64)
    scale = np.sqrt(np.outer((a.astype(np.float64) ** 2).sum(0), (b.astype(np.float64) ** 2).sum(0)))
    for prec, tol in ((L.GRAM_F64, 1e-13), (L.GRAM_F32, 2e-6), (L.GRAM_BF16X3, 2e-5)):
        Gn = noalloc(da, db, prec)
        Gc = c2.gram(da, db, prec=prec).cpu().numpy()
        assert np.max(np.abs(Gn - ref) / scale) <= tol, prec
        assert np.max(np.abs(Gn - Gc) / scale) <= 2 * tol, prec
    c2.close()
    # 3) FP64 data, smaller still (one workgroup)
    n3 = 1000
    A3 = synth.random_sym(n3, 2, seed=4)
    c3 = upload(A3, False)
    a = synth.gaussian_block(n3, 5, seed=5)
    da = to_dev(a, np.float64)
    Gn = noalloc(da, da, L.GRAM_AUTO, f32=False)
    Gc = c3.gram(da, da).cpu().numpy()
    ref = a.T @ a
    scale = np.sqrt(np.outer((a ** 2).sum(0), (a ** 2).sum(0)))
    assert np.max(np.abs(Gn - ref) / scale) <= 1e-13
    assert np.max(np.abs(Gn - Gc) / scale) <= 2e-13
    c3.close()


def test_noalloc_gram_rejects_sizes_beyond_scratch():
    import paper_2109_00485_amd as L
    torch = torch_cuda()
    lib = L.load()
    a = torch.zeros((64, 49), dtype=torch.float32, device="cuda")
    G = torch.zeros((49, 49), dtype=torch.float64, device="cuda")
    p = lambda t: ctypes.c_void_p(t.data_ptr())
    assert lib.lobpcg_gram_noalloc(p(a), 49, p(a), 49, 64, L.F32, p(G), L.GRAM_F64, None) == L.EUNSUPPORTED
    assert lib.lobpcg_gram_noalloc(p(a), 8, p(a), 8, 0, L.F32, p(G), L.GRAM_F64, None) == L.EINVAL
    assert lib.lobpcg_gram_noalloc(p(a), 8, p(a), 8, 64, L.F64, p(G), L.GRAM_F32, None) == L.EINVAL
    assert lib.lobpcg_gram_noalloc(None, 8, p(a), 8, 64, L.F32, p(G), L.GRAM_F64, None) == L.EINVAL
