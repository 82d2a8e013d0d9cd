"""Seeded synthetic inputs shared by the FP64 oracle and the HIP path.

This package only *generates* matrices and vector blocks; it holds none of
the solver's arithmetic.  The heavy lifting is a small C library
(``synth.c``) built with gcc/OpenMP; every draw is a pure function of
(seed, stream, counter), so outputs are identical for any thread count.

Matrices are the upper triangle (diagonal included) of a symmetric H, in CSR
with ascending columns and the diagonal first in each row.  The workload
presets in :mod:`synth.workloads` stand in for the paper's nuclear CI
Hamiltonians (Table 2), which are not available: half-stored symmetric,
sparse, and (for the tiled family) made of sparse tiles as described in the
paper's section on local SpMM.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import weakref

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "synth.c")
_LIB = os.path.join(_HERE, "libsynth.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile ``libsynth.so`` in place with gcc."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O3", "-fopenmp", "-fPIC", "-shared", "-Wall",
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB):
        build(force=True)
    lib = ctypes.CDLL(_LIB)
    P = ctypes.c_void_p
    i64, u64, dbl, cint = ctypes.c_int64, ctypes.c_uint64, ctypes.c_double, ctypes.c_int
    lib.synth_rs.restype = P
    lib.synth_rs.argtypes = [i64, i64, u64, dbl, dbl, cint]
    lib.synth_tiled.restype = P
    lib.synth_tiled.argtypes = [i64, i64, i64, dbl, u64, dbl, dbl, cint]
    lib.synth_zipf.restype = P
    lib.synth_zipf.argtypes = [i64, dbl, i64, i64, u64, dbl, dbl, cint]
    for name in ("synth_csr_n", "synth_csr_nnz"):
        getattr(lib, name).restype = i64
        getattr(lib, name).argtypes = [P]
    for name in ("synth_csr_row_ptr", "synth_csr_col", "synth_csr_val", "synth_csr_diag"):
        getattr(lib, name).restype = P
        getattr(lib, name).argtypes = [P]
    lib.synth_csr_is_f32.restype = cint
    lib.synth_csr_is_f32.argtypes = [P]
    lib.synth_csr_free.restype = None
    lib.synth_csr_free.argtypes = [P]
    lib.synth_gaussian_block.restype = None
    lib.synth_gaussian_block.argtypes = [i64, i64, u64, P]
    lib.synth_gaussian_block_f32.restype = None
    lib.synth_gaussian_block_f32.argtypes = [i64, i64, u64, P]
    lib.synth_sorted_uniform.restype = None
    lib.synth_sorted_uniform.argtypes = [i64, u64, dbl, P]
    _lib = lib
    return lib


class UpperCSR:
    """Upper triangle of a symmetric matrix in CSR (views onto C-owned memory).

    Attributes: ``n``, ``nnz``, ``row_ptr`` (int64, n+1), ``col`` (int32),
    ``val`` (float64 or float32), ``diag`` (float64, equal to the stored
    diagonal values).
    """

    def __init__(self, handle, desc: str = ""):
        if not handle:
            raise ValueError("synth: invalid generator parameters")
        lib = _load()
        self._h = handle
        self.n = int(lib.synth_csr_n(handle))
        self.nnz = int(lib.synth_csr_nnz(handle))
        f32 = bool(lib.synth_csr_is_f32(handle))
        self.desc = desc

        def view(ptr, count, ctype, dtype):
            if count == 0:
                return np.zeros(0, dtype=dtype)
            arr = np.ctypeslib.as_array(ctypes.cast(ptr, ctypes.POINTER(ctype)), shape=(count,))
            return arr.view(dtype)

        self.row_ptr = view(lib.synth_csr_row_ptr(handle), self.n + 1, ctypes.c_int64, np.int64)
        self.col = view(lib.synth_csr_col(handle), self.nnz, ctypes.c_int32, np.int32)
        if f32:
            self.val = view(lib.synth_csr_val(handle), self.nnz, ctypes.c_float, np.float32)
        else:
            self.val = view(lib.synth_csr_val(handle), self.nnz, ctypes.c_double, np.float64)
        self.diag = view(lib.synth_csr_diag(handle), self.n, ctypes.c_double, np.float64)
        self._fin = weakref.finalize(self, lib.synth_csr_free, handle)

    @property
    def dtype(self):
        return self.val.dtype

    def row_lengths(self) -> np.ndarray:
        return np.diff(self.row_ptr)

    def free(self):
        self.row_ptr = self.col = self.val = self.diag = None
        self._fin()


class ArrayCSR:
    """Upper-triangle CSR built from NumPy arrays (small structured cases)."""

    def __init__(self, n, row_ptr, col, val, desc: str = ""):
        self.n = int(n)
        self.row_ptr = np.ascontiguousarray(row_ptr, dtype=np.int64)
        self.col = np.ascontiguousarray(col, dtype=np.int32)
        self.val = np.ascontiguousarray(val)
        self.nnz = int(self.row_ptr[-1])
        self.desc = desc
        d = np.zeros(self.n)
        for i in range(self.n):
            b, e = self.row_ptr[i], self.row_ptr[i + 1]
            hit = np.nonzero(self.col[b:e] == i)[0]
            if hit.size:
                d[i] = float(self.val[b + hit[0]])
        self.diag = d

    @property
    def dtype(self):
        return self.val.dtype

    def row_lengths(self) -> np.ndarray:
        return np.diff(self.row_ptr)

    def free(self):
        pass


def random_sym(n: int, draws: int, seed: int, dmax: float = 200.0, scale: float = 0.5,
               f32: bool = False) -> UpperCSR:
    """Each row draws ``draws`` distinct partners; values N(0,1)*scale are summed
    into the symmetric pair; d = sort(U[0, dmax))."""
    lib = _load()
    return UpperCSR(lib.synth_rs(n, draws, seed, dmax, scale, int(f32)),
                    desc=f"random_sym(n={n},draws={draws},seed={seed})")


def tiled(n: int, tile: int = 64, tile_draws: int = 47, p: float = 400.0 / (64 * 95),
          seed: int = 0, dmax: float = 500.0, scale: float = 0.1, f32: bool = True) -> UpperCSR:
    """Block-sparse pattern of ``tile`` x ``tile`` sparse tiles: each tile-row draws
    ``tile_draws`` distinct tile columns (pattern symmetrised), each present tile
    entry is kept with probability ``p`` and valued N(0,1)*scale."""
    lib = _load()
    return UpperCSR(lib.synth_tiled(n, tile, tile_draws, p, seed, dmax, scale, int(f32)),
                    desc=f"tiled(n={n},tile={tile},draws={tile_draws},p={p:.4g},seed={seed})")


def zipf(n: int, a: float = 1.5, lmin: int = 20, lmax: int = 20000, seed: int = 0,
         dmax: float = 1000.0, scale: float = 0.05, f32: bool = True) -> UpperCSR:
    """Power-law full-row degrees clip(Zipf(a), lmin, lmax); row i draws ceil(L_i/2)
    partners with probability proportional to their degree."""
    lib = _load()
    return UpperCSR(lib.synth_zipf(n, a, lmin, lmax, seed, dmax, scale, int(f32)),
                    desc=f"zipf(n={n},a={a},seed={seed})")


def gaussian_block(n: int, k: int, seed: int, dtype=np.float64) -> np.ndarray:
    """n x k row-major block of N(0,1) draws (stream ``seed``)."""
    lib = _load()
    if np.dtype(dtype) == np.float32:
        out = np.empty((n, k), dtype=np.float32)
        lib.synth_gaussian_block_f32(n, k, seed, out.ctypes.data)
    else:
        out = np.empty((n, k), dtype=np.float64)
        lib.synth_gaussian_block(n, k, seed, out.ctypes.data)
    return out


def sorted_uniform(n: int, seed: int, dmax: float) -> np.ndarray:
    lib = _load()
    out = np.empty(n, dtype=np.float64)
    lib.synth_sorted_uniform(n, seed, dmax, out.ctypes.data)
    return out


# ---------------- small structured matrices with known spectra ----------------

def laplacian_1d(n: int, dtype=np.float64) -> ArrayCSR:
    """tridiag(-1, 2, -1), upper triangle."""
    rp = [0]
    col, val = [], []
    for i in range(n):
        col.append(i); val.append(2.0)
        if i + 1 < n:
            col.append(i + 1); val.append(-1.0)
        rp.append(len(col))
    return ArrayCSR(n, rp, col, np.asarray(val, dtype=dtype), desc=f"laplacian_1d({n})")


def diagonal(d, dtype=np.float64) -> ArrayCSR:
    d = np.asarray(d, dtype=np.float64)
    n = d.size
    return ArrayCSR(n, np.arange(n + 1), np.arange(n), d.astype(dtype), desc=f"diagonal({n})")


def blocks_2x2(a, b, c, dtype=np.float64) -> ArrayCSR:
    """Direct sum of [[a_q, b_q], [b_q, c_q]] blocks."""
    a, b, c = (np.asarray(x, dtype=np.float64) for x in (a, b, c))
    m = a.size
    rp = [0]
    col, val = [], []
    for q in range(m):
        i = 2 * q
        col += [i, i + 1]; val += [a[q], b[q]]; rp.append(len(col))
        col += [i + 1]; val += [c[q]]; rp.append(len(col))
    return ArrayCSR(2 * m, rp, col, np.asarray(val, dtype=dtype), desc=f"blocks_2x2({m})")


def from_dense_upper(A: np.ndarray, dtype=None) -> ArrayCSR:
    """Upper-triangle CSR of a dense symmetric matrix (diagonal always stored)."""
    A = np.asarray(A)
    n = A.shape[0]
    rp = [0]
    col, val = [], []
    for i in range(n):
        col.append(i); val.append(A[i, i])
        for j in range(i + 1, n):
            if A[i, j] != 0:
                col.append(j); val.append(A[i, j])
        rp.append(len(col))
    return ArrayCSR(n, rp, col, np.asarray(val, dtype=dtype or A.dtype), desc=f"dense({n})")


def near_diagonal(n: int = 2000, draws: int = 10, seed: int = 3, coupling: float = 0.01, dtype=np.float64) -> ArrayCSR:
    """Diagonal 1.0, 1.1, 1.2, ... plus weak random couplings N(0,1) * coupling
    between each row and `draws` random partners (pairs summed): eigenvalues
    ~0.1 apart, each close to one diagonal entry."""
    import scipy.sparse as sp
    rng = np.random.default_rng(seed)
    r = np.repeat(np.arange(n), draws)
    c = rng.integers(0, n, n * draws)
    keep = r != c
    i, j = np.minimum(r, c)[keep], np.maximum(r, c)[keep]
    v = rng.standard_normal(i.size) * coupling
    U = sp.coo_matrix((v, (i, j)), shape=(n, n)).tocsr()
    U.sum_duplicates()
    U = (U + sp.diags(1.0 + 0.1 * np.arange(n))).tocsr()
    U.sort_indices()
    return ArrayCSR(n, U.indptr, U.indices, U.data.astype(dtype), desc=f"near_diagonal({n})")
