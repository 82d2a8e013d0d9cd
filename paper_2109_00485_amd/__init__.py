"""MI355X (gfx950) LOBPCG hot path: Python binding of the C ABI in include/lobpcg.h.

This module only marshals arguments: torch CUDA tensors supply device memory
(``data_ptr``) and streams (``cuda_stream``); every step of the computation
runs in the HIP kernels of ``liblobpcg.so``.  If the library has not been
built, importing works but every call raises -- there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass, field
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liblobpcg.so")

OK, EINVAL, ENOMEM, EHIP, ENOTSPD, ENOCONV, ENONFINITE, EUNSUPPORTED = 0, -1, -2, -3, -4, -5, -6, -7
F32, F64 = 1, 2
GRAM_AUTO, GRAM_F64, GRAM_F32, GRAM_BF16X3 = 0, 1, 2, 3
PRECOND_NONE, PRECOND_DIAG, PRECOND_MLP = 0, 1, 2
FORMAT_AUTO, FORMAT_CSR, FORMAT_TILED = 0, 1, 2


class LobpcgError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"[{status}] {msg}")
        self.status = status


class Opts(ctypes.Structure):
    _fields_ = [("dtype", ctypes.c_int), ("gram", ctypes.c_int), ("format", ctypes.c_int),
                ("tile", ctypes.c_int), ("kmax", ctypes.c_int), ("tau_rel", ctypes.c_double),
                ("eps_rel", ctypes.c_double)]


class Info(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int), ("n_spmm", ctypes.c_int), ("p_dropped", ctypes.c_int),
                ("cholqr_retries", ctypes.c_int), ("confirmations", ctypes.c_int), ("refreshes", ctypes.c_int),
                ("status", ctypes.c_int),
                ("gamma", ctypes.c_double),
                ("theta_hist", ctypes.POINTER(ctypes.c_double)), ("rel_hist", ctypes.POINTER(ctypes.c_double)),
                ("timing", ctypes.c_int),
                ("t_spmm", ctypes.c_double), ("t_precond_update", ctypes.c_double), ("t_gram", ctypes.c_double),
                ("t_rr", ctypes.c_double), ("t_orth", ctypes.c_double), ("t_total", ctypes.c_double)]


_lib = None


def load(path: str = LIB_PATH):
    """Load liblobpcg.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with paper_2109_00485_amd.build.build() "
                           "(there is no CPU fallback)")
    lib = ctypes.CDLL(path)
    P, i64, cint, dbl = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int, ctypes.c_double
    lib.lobpcg_opts_default.restype = None
    lib.lobpcg_opts_default.argtypes = [ctypes.POINTER(Opts)]
    lib.lobpcg_create.restype = cint
    lib.lobpcg_create.argtypes = [ctypes.POINTER(P), i64, P, P, P, ctypes.POINTER(Opts), P]
    lib.lobpcg_destroy.restype = None
    lib.lobpcg_destroy.argtypes = [P]
    lib.lobpcg_spmm_sym.restype = cint
    lib.lobpcg_spmm_sym.argtypes = [P, P, P, cint, P]
    lib.lobpcg_precond_apply.restype = cint
    lib.lobpcg_precond_apply.argtypes = [P, P, P, P, cint, cint, P]
    lib.lobpcg_gram.restype = cint
    lib.lobpcg_gram.argtypes = [P, P, cint, P, cint, P, cint, P]
    lib.lobpcg_solve.restype = cint
    lib.lobpcg_solve.argtypes = [P, cint, cint, P, P, P, dbl, cint, cint, ctypes.POINTER(Info), P]
    lib.lobpcg_query.restype = cint
    lib.lobpcg_query.argtypes = [P, ctypes.POINTER(i64), ctypes.POINTER(i64), ctypes.POINTER(cint),
                                 ctypes.POINTER(cint), ctypes.POINTER(dbl)]
    lib.lobpcg_get_diag.restype = cint
    lib.lobpcg_get_diag.argtypes = [P, P, P]
    lib.lobpcg_strerror.restype = ctypes.c_char_p
    lib.lobpcg_strerror.argtypes = [cint]
    lib.lobpcg_last_error.restype = ctypes.c_char_p
    lib.lobpcg_last_error.argtypes = [P]
    _lib = lib
    return lib


def default_opts() -> Opts:
    o = Opts()
    load().lobpcg_opts_default(ctypes.byref(o))
    return o


def _stream_ptr(stream=None):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _dev_ptr(t, dtype=None, name="tensor"):
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA (HIP) torch tensor")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous (row-major)")
    if dtype is not None and t.dtype != dtype:
        raise TypeError(f"{name} must have dtype {dtype}, got {t.dtype}")
    return ctypes.c_void_p(t.data_ptr())


@dataclass
class SolveResult:
    evals: np.ndarray
    rel: np.ndarray
    status: int
    iters: int
    n_spmm: int
    p_dropped: int
    cholqr_retries: int
    confirmations: int
    refreshes: int
    gamma: float
    times: dict = field(default_factory=dict)
    theta_hist: Optional[np.ndarray] = None
    rel_hist: Optional[np.ndarray] = None


class Context:
    """A matrix H (upper triangle in CSR, device-resident) and its workspaces."""

    def __init__(self, n, row_ptr, col, val, *, dtype=None, gram=GRAM_AUTO, fmt=FORMAT_AUTO, kmax=16,
                 tau_rel=1e-3, eps_rel=1e-5, stream=None):
        import torch
        lib = load()
        if dtype is None:
            dtype = F64 if val.dtype == torch.float64 else F32
        tval = torch.float64 if dtype == F64 else torch.float32
        o = default_opts()
        o.dtype, o.gram, o.format, o.kmax = dtype, gram, fmt, kmax
        o.tau_rel, o.eps_rel = tau_rel, eps_rel
        h = ctypes.c_void_p()
        rc = lib.lobpcg_create(ctypes.byref(h), int(n), _dev_ptr(row_ptr, torch.int64, "row_ptr"),
                               _dev_ptr(col, torch.int32, "col"), _dev_ptr(val, tval, "val"), ctypes.byref(o),
                               _stream_ptr(stream))
        if rc != OK:
            raise LobpcgError(rc, lib.lobpcg_strerror(rc).decode())
        self._h = h
        self.n = int(n)
        self.dtype = dtype
        self.torch_dtype = tval
        self.kmax = kmax

    @classmethod
    def from_csr(cls, A, device="cuda", **kw):
        """Upload an upper-triangle CSR (numpy arrays ``row_ptr, col, val``)."""
        import torch
        rp = torch.from_numpy(np.ascontiguousarray(A.row_ptr, dtype=np.int64)).to(device)
        ci = torch.from_numpy(np.ascontiguousarray(A.col, dtype=np.int32)).to(device)
        va = torch.from_numpy(np.ascontiguousarray(A.val)).to(device)
        ctx = cls(A.n, rp, ci, va, **kw)
        torch.cuda.synchronize()
        del rp, ci, va
        return ctx

    # -- helpers ---------------------------------------------------------------------------
    def _check(self, rc, what):
        if rc != OK:
            msg = load().lobpcg_last_error(self._h).decode()
            raise LobpcgError(rc, f"{what}: {msg or load().lobpcg_strerror(rc).decode()}")

    def close(self):
        if getattr(self, "_h", None):
            load().lobpcg_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def query(self) -> dict:
        n, nnz, fmt, dt, g = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int(), ctypes.c_int(), ctypes.c_double()
        self._check(load().lobpcg_query(self._h, ctypes.byref(n), ctypes.byref(nnz), ctypes.byref(fmt),
                                        ctypes.byref(dt), ctypes.byref(g)), "query")
        return dict(n=n.value, nnz=nnz.value, format=fmt.value, dtype=dt.value, gamma=g.value)

    def diag(self, stream=None):
        import torch
        d = torch.empty(self.n, dtype=self.torch_dtype, device="cuda")
        self._check(load().lobpcg_get_diag(self._h, _dev_ptr(d), _stream_ptr(stream)), "get_diag")
        return d

    # -- the five calls --------------------------------------------------------------------
    def spmm_sym(self, X, Y=None, stream=None):
        import torch
        k = X.shape[1]
        if Y is None:
            Y = torch.empty_like(X)
        self._check(load().lobpcg_spmm_sym(self._h, _dev_ptr(X, self.torch_dtype, "X"),
                                           _dev_ptr(Y, self.torch_dtype, "Y"), k, _stream_ptr(stream)),
                    "spmm_sym")
        return Y

    def precond_apply(self, R, theta, W=None, kind=PRECOND_DIAG, stream=None):
        import torch
        if W is None:
            W = torch.empty_like(R)
        self._check(load().lobpcg_precond_apply(self._h, _dev_ptr(R, self.torch_dtype, "R"),
                                                _dev_ptr(theta, torch.float64, "theta"),
                                                _dev_ptr(W, self.torch_dtype, "W"), R.shape[1], kind,
                                                _stream_ptr(stream)), "precond_apply")
        return W

    def gram(self, A, B, prec=GRAM_AUTO, G=None, stream=None):
        import torch
        ka, kb = A.shape[1], B.shape[1]
        if G is None:
            G = torch.empty((ka, kb), dtype=torch.float64, device=A.device)
        self._check(load().lobpcg_gram(self._h, _dev_ptr(A, self.torch_dtype, "A"), ka,
                                       _dev_ptr(B, self.torch_dtype, "B"), kb,
                                       _dev_ptr(G, torch.float64, "G"), prec, _stream_ptr(stream)), "gram")
        return G

    def solve(self, X, nev, tol=1e-6, maxiter=5000, precond=PRECOND_DIAG, history=False, timing=False,
              stream=None, raise_on_noconv=False) -> SolveResult:
        k = X.shape[1]
        evals = np.zeros(k)
        rel = np.zeros(k)
        info = Info()
        th = rh = None
        if history:
            th = np.zeros(max(maxiter, 1) * k)
            rh = np.zeros(max(maxiter, 1) * k)
            info.theta_hist = th.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
            info.rel_hist = rh.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        info.timing = int(bool(timing))
        rc = load().lobpcg_solve(self._h, k, nev, _dev_ptr(X, self.torch_dtype, "X"),
                                 evals.ctypes.data_as(ctypes.c_void_p), rel.ctypes.data_as(ctypes.c_void_p),
                                 float(tol), int(maxiter), int(precond), ctypes.byref(info), _stream_ptr(stream))
        if rc not in (OK, ENOCONV) or (rc == ENOCONV and raise_on_noconv):
            self._check(rc, "solve")
        res = SolveResult(evals=evals, rel=rel, status=rc, iters=info.iters, n_spmm=info.n_spmm,
                          p_dropped=info.p_dropped, cholqr_retries=info.cholqr_retries,
                          confirmations=info.confirmations, refreshes=info.refreshes, gamma=info.gamma,
                          times=dict(spmm=info.t_spmm, precond_update=info.t_precond_update, gram=info.t_gram,
                                     rr=info.t_rr, orth=info.t_orth, total=info.t_total))
        if history:
            res.theta_hist = th.reshape(-1, k)[:info.iters]
            res.rel_hist = rh.reshape(-1, k)[:info.iters]
        return res
