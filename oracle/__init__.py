"""FP64 CPU oracle for the symmetric-SpMM / LOBPCG hot path.

TEST INFRASTRUCTURE ONLY.  Nothing in the product library imports, links or
calls this package; only the tests, the smoke check and the CPU-baseline leg
of the benchmark do.  It shares no code with the HIP path: its sparse
product is plain C loops (``spmm.c``), its dense algebra is NumPy/LAPACK, and
it follows the paper's algorithm step by step in double precision.

Modules
  oracle (this file)   FP64 symmetric SpMM from the upper triangle (C, OpenMP)
  oracle.dense         Cholesky QR, Gram blocks, Rayleigh-Ritz (NumPy/LAPACK)
  oracle.lobpcg        Algorithm 1 in FP64, with the readings of the paper
  oracle.precond       diagonal shift-inverse preconditioner
  oracle.mlp           learned-preconditioner network: forward, backward, Adam
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import weakref

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "spmm.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile ``liboracle.so`` in place with gcc (building the checker is not using it)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-Wall",
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB):
        build(force=True)
    # idle OpenMP workers must not spin against the BLAS thread pool
    os.environ.setdefault("OMP_WAIT_POLICY", "PASSIVE")
    lib = ctypes.CDLL(_LIB)
    P, i64, cint = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int
    lib.oracle_mat_create.restype = P
    lib.oracle_mat_create.argtypes = [i64, P, P, P, cint]
    lib.oracle_mat_free.restype = None
    lib.oracle_mat_free.argtypes = [P]
    for name in ("oracle_spmm", "oracle_spmm_abs"):
        getattr(lib, name).restype = None
        getattr(lib, name).argtypes = [P, i64, P, P]
    lib.oracle_spmm_rows.restype = None
    lib.oracle_spmm_rows.argtypes = [P, i64, P, i64, P, P, P]
    lib.oracle_gershgorin.restype = ctypes.c_double
    lib.oracle_gershgorin.argtypes = [P]
    lib.oracle_row_offdiag_abs.restype = None
    lib.oracle_row_offdiag_abs.argtypes = [P, P]
    lib.oracle_row_offdiag_count.restype = None
    lib.oracle_row_offdiag_count.argtypes = [P, P]
    lib.oracle_set_threads.restype = None
    lib.oracle_set_threads.argtypes = [cint]
    lib.oracle_get_threads.restype = cint
    lib.oracle_get_threads.argtypes = []
    _lib = lib
    return lib


def threads() -> int:
    """Threads the oracle's OpenMP loops use."""
    return int(_load().oracle_get_threads())


def set_threads(t: int) -> None:
    """Set the threads of the oracle's OpenMP loops (baseline timing only)."""
    _load().oracle_set_threads(int(t))


class SymMatrix:
    """Symmetric H held as its upper triangle U (FP64 copy, plus a CSC copy of the
    strict upper part for the transposed pass)."""

    def __init__(self, n, row_ptr, col, val):
        lib = _load()
        self.n = int(n)
        rp = np.ascontiguousarray(row_ptr, dtype=np.int64)
        ci = np.ascontiguousarray(col, dtype=np.int32)
        val = np.ascontiguousarray(val)
        if val.dtype == np.float32:
            f32 = 1
        else:
            val = np.ascontiguousarray(val, dtype=np.float64)
            f32 = 0
        if rp.shape[0] != self.n + 1 or ci.shape[0] != rp[-1] or val.shape[0] != rp[-1]:
            raise ValueError("oracle: inconsistent CSR arrays")
        self.nnz = int(rp[-1])
        h = lib.oracle_mat_create(self.n, rp.ctypes.data, ci.ctypes.data, val.ctypes.data, f32)
        if not h:
            raise MemoryError("oracle_mat_create failed")
        self._h = h
        self._fin = weakref.finalize(self, lib.oracle_mat_free, h)

    @classmethod
    def from_csr(cls, A):
        """From any object with ``n, row_ptr, col, val`` (e.g. a synth matrix)."""
        return cls(A.n, A.row_ptr, A.col, A.val)

    def matmul(self, X: np.ndarray) -> np.ndarray:
        """Y = H X in FP64 (X is upcast exactly if it is FP32)."""
        X = np.ascontiguousarray(X, dtype=np.float64)
        squeeze = X.ndim == 1
        if squeeze:
            X = X[:, None]
        if X.shape[0] != self.n:
            raise ValueError("oracle: X has wrong number of rows")
        Y = np.empty_like(X)
        _load().oracle_spmm(self._h, X.shape[1], X.ctypes.data, Y.ctypes.data)
        return Y[:, 0] if squeeze else Y

    __matmul__ = matmul

    def abs_matmul(self, X: np.ndarray) -> np.ndarray:
        """|H| |X| in FP64: the magnitude scale of each output entry's summands."""
        X = np.ascontiguousarray(X, dtype=np.float64)
        Y = np.empty_like(X)
        _load().oracle_spmm_abs(self._h, X.shape[1], X.ctypes.data, Y.ctypes.data)
        return Y

    def rows(self, X: np.ndarray, rows) -> tuple[np.ndarray, np.ndarray]:
        """(H X)[rows] and (|H||X|)[rows], computed row by row."""
        X = np.ascontiguousarray(X, dtype=np.float64)
        rows = np.ascontiguousarray(rows, dtype=np.int64)
        k = X.shape[1]
        Y = np.empty((rows.size, k))
        Ya = np.empty((rows.size, k))
        _load().oracle_spmm_rows(self._h, k, X.ctypes.data, rows.size, rows.ctypes.data,
                                 Y.ctypes.data, Ya.ctypes.data)
        return Y, Ya

    def gershgorin(self) -> float:
        return float(_load().oracle_gershgorin(self._h))

    def row_offdiag_abs(self) -> np.ndarray:
        out = np.empty(self.n)
        _load().oracle_row_offdiag_abs(self._h, out.ctypes.data)
        return out

    def row_offdiag_count(self) -> np.ndarray:
        out = np.empty(self.n, dtype=np.int64)
        _load().oracle_row_offdiag_count(self._h, out.ctypes.data)
        return out
