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
GRAM_AUTO, GRAM_F64, GRAM_F32, GRAM_BF16X3, GRAM_BF16X6 = 0, 1, 2, 3, 4
PRECOND_NONE, PRECOND_DIAG, PRECOND_MLP, PRECOND_FOM = 0, 1, 2, 3
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
                ("t_rr", ctypes.c_double), ("t_orth", ctypes.c_double), ("t_total", ctypes.c_double),
                ("harvest", ctypes.c_void_p), ("cholqr_shifted", ctypes.c_int), ("mlp_fallbacks", ctypes.c_longlong),
                ("locked_max", ctypes.c_int)]


MLP_NIN, MLP_HID, MLP_NPARAM, MLP_NBLOB = 4, 64, 4545, 4553
# blob layout: (name, shape) in order
MLP_LAYOUT = (("W1", (64, 4)), ("b1", (64,)), ("W2", (64, 64)), ("b2", (64,)), ("w3", (64,)), ("b3", ()),
              ("mu", (4,)), ("sigma", (4,)))


class Harvest(ctypes.Structure):
    _fields_ = [("every", ctypes.c_int), ("rows", ctypes.c_int), ("nev", ctypes.c_int),
                ("xstar", ctypes.c_void_p), ("seed", ctypes.c_uint64), ("capacity", ctypes.c_int64),
                ("capacity_groups", ctypes.c_int), ("feat", ctypes.c_void_p), ("U", ctypes.c_void_p),
                ("T", ctypes.c_void_p), ("w", ctypes.c_void_p), ("Xrow", ctypes.c_void_p),
                ("row", ctypes.c_void_p), ("group_off", ctypes.c_void_p), ("nsamples", ctypes.c_int64),
                ("ngroups", ctypes.c_int), ("full", ctypes.c_int)]


class MlpBatch(ctypes.Structure):
    _fields_ = [("nsamples", ctypes.c_int64), ("ngroups", ctypes.c_int), ("k", ctypes.c_int),
                ("feat", ctypes.c_void_p), ("U", ctypes.c_void_p), ("T", ctypes.c_void_p),
                ("w", ctypes.c_void_p), ("Xrow", ctypes.c_void_p), ("group_off", ctypes.c_void_p)]


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
    lib.lobpcg_create_rp32.restype = cint
    lib.lobpcg_create_rp32.argtypes = [ctypes.POINTER(P), i64, P, P, P, ctypes.POINTER(Opts), P]
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
    fptr = ctypes.POINTER(ctypes.c_float)
    lib.lobpcg_mlp_create.restype = cint
    lib.lobpcg_mlp_create.argtypes = [ctypes.POINTER(P), fptr]
    lib.lobpcg_mlp_destroy.restype = None
    lib.lobpcg_mlp_destroy.argtypes = [P]
    lib.lobpcg_mlp_set_params.restype = cint
    lib.lobpcg_mlp_set_params.argtypes = [P, fptr]
    lib.lobpcg_mlp_get_params.restype = cint
    lib.lobpcg_mlp_get_params.argtypes = [P, fptr]
    lib.lobpcg_mlp_last_error.restype = ctypes.c_char_p
    lib.lobpcg_mlp_last_error.argtypes = [P]
    lib.lobpcg_set_mlp.restype = cint
    lib.lobpcg_set_mlp.argtypes = [P, P]
    lib.lobpcg_set_cholqr_passes.restype = cint
    lib.lobpcg_set_cholqr_passes.argtypes = [P, cint]
    lib.lobpcg_set_soft_lock.restype = cint
    lib.lobpcg_set_soft_lock.argtypes = [P, cint]
    lib.lobpcg_cholqr.restype = cint
    lib.lobpcg_cholqr.argtypes = [P, P, cint, cint, ctypes.POINTER(cint), P]
    lib.lobpcg_orthonormalize.restype = cint
    lib.lobpcg_orthonormalize.argtypes = [P, P, P, cint, ctypes.POINTER(cint), P]
    lib.lobpcg_set_fom_steps.restype = cint
    lib.lobpcg_set_fom_steps.argtypes = [P, cint]
    lib.lobpcg_set_test_faults.restype = cint
    lib.lobpcg_set_test_faults.argtypes = [P, cint, cint]
    lib.lobpcg_set_precond_offset.restype = cint
    lib.lobpcg_set_precond_offset.argtypes = [P, dbl]
    lib.lobpcg_get_features.restype = cint
    lib.lobpcg_get_features.argtypes = [P, P, P, P]
    lib.lobpcg_mlp_forward.restype = cint
    lib.lobpcg_mlp_forward.argtypes = [P, P, i64, P, P]
    lib.lobpcg_mlp_fit_standardizer.restype = cint
    lib.lobpcg_mlp_fit_standardizer.argtypes = [P, P, i64, P]
    lib.lobpcg_mlp_loss_grad.restype = cint
    lib.lobpcg_mlp_loss_grad.argtypes = [P, ctypes.POINTER(MlpBatch), ctypes.POINTER(dbl), fptr, P]
    lib.lobpcg_mlp_train_step.restype = cint
    lib.lobpcg_mlp_train_step.argtypes = [P, ctypes.POINTER(MlpBatch), ctypes.c_float, ctypes.POINTER(dbl), P]
    lib.lobpcg_harvest_block.restype = cint
    lib.lobpcg_harvest_block.argtypes = [P, P, P, P, cint, ctypes.POINTER(Harvest), P]
    lib.lobpcg_gram_noalloc.restype = cint
    lib.lobpcg_gram_noalloc.argtypes = [P, cint, P, cint, i64, cint, P, cint, P]
    lib.lobpcg_stream_probe.restype = cint
    lib.lobpcg_stream_probe.argtypes = [cint, P, P, i64, P]
    _lib = lib
    return lib


PROBE_READ, PROBE_WRITE, PROBE_COPY = 0, 1, 2
FAULT_CHOLQR_SHIFT, FAULT_CHOLQR_ONCE, FAULT_CHOLQR_ALWAYS, FAULT_RR_DROP_P, FAULT_RR = 1, 2, 4, 8, 16


def stream_probe(op, a, b, nbytes, stream=None):
    """lobpcg_stream_probe: plain read / write / copy of ``nbytes`` on the device
    (a, b: CUDA tensors, 16-byte aligned)."""
    rc = load().lobpcg_stream_probe(int(op), ctypes.c_void_p(a.data_ptr()) if a is not None else None,
                                    ctypes.c_void_p(b.data_ptr()) if b is not None else None, int(nbytes),
                                    _stream_ptr(stream))
    if rc != OK:
        raise LobpcgError(rc, "stream_probe: " + load().lobpcg_strerror(rc).decode())


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
    cholqr_shifted: int = 0
    mlp_fallbacks: int = 0
    locked_max: int = 0
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
        # int32 row offsets go through lobpcg_create_rp32, int64 through lobpcg_create
        create, rpt = ((lib.lobpcg_create_rp32, torch.int32) if row_ptr.dtype == torch.int32
                       else (lib.lobpcg_create, torch.int64))
        rc = create(ctypes.byref(h), int(n), _dev_ptr(row_ptr, rpt, "row_ptr"),
                    _dev_ptr(col, torch.int32, "col"), _dev_ptr(val, tval, "val"), ctypes.byref(o),
                    _stream_ptr(stream))
        if rc != OK:
            raise LobpcgError(rc, lib.lobpcg_strerror(rc).decode())
        self._h = h
        self.n = int(n)
        self.dtype = dtype
        self.torch_dtype = tval
        self.kmax = kmax
        self.precond_offset = 0.0

    @classmethod
    def from_csr(cls, A, device="cuda", **kw):
        """Upload an upper-triangle CSR (numpy arrays ``row_ptr, col, val``);
        int32 row offsets stay int32 (lobpcg_create_rp32), others are int64."""
        import torch
        rpd = np.int32 if np.asarray(A.row_ptr).dtype == np.int32 else np.int64
        rp = torch.from_numpy(np.ascontiguousarray(A.row_ptr, dtype=rpd)).to(device)
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

    def set_cholqr_passes(self, passes: int):
        """lobpcg_set_cholqr_passes: 1 (Cholesky QR) or 2 (CholeskyQR2) in solves."""
        self._check(load().lobpcg_set_cholqr_passes(self._h, int(passes)), "set_cholqr_passes")

    def set_soft_lock(self, on: bool):
        """lobpcg_set_soft_lock: converged columns leave W and P in solves."""
        self._check(load().lobpcg_set_soft_lock(self._h, int(bool(on))), "set_soft_lock")

    def cholqr(self, W, passes=1, stream=None):
        """lobpcg_cholqr: W <- its Cholesky QR factor Q, in place; returns the number of
        shifted passes."""
        sh = ctypes.c_int()
        self._check(load().lobpcg_cholqr(self._h, _dev_ptr(W, self.torch_dtype, "W"), W.shape[1], int(passes),
                                         ctypes.byref(sh), _stream_ptr(stream)), "cholqr")
        return sh.value

    def orthonormalize(self, X, W, stream=None):
        """lobpcg_orthonormalize: W <- Cholesky QR of W - X (X^T W), in place; returns 1
        when the shifted factorisation was used."""
        sh = ctypes.c_int()
        self._check(load().lobpcg_orthonormalize(self._h, _dev_ptr(X, self.torch_dtype, "X"),
                                                 _dev_ptr(W, self.torch_dtype, "W"), W.shape[1],
                                                 ctypes.byref(sh), _stream_ptr(stream)), "orthonormalize")
        return sh.value

    def set_fom_steps(self, m: int):
        """lobpcg_set_fom_steps: FOM steps of the block-diagonal preconditioner (1..8)."""
        self._check(load().lobpcg_set_fom_steps(self._h, int(m)), "set_fom_steps")

    def set_test_faults(self, mask: int, iteration: int = 1):
        """lobpcg_set_test_faults: force the solver's failure branches at one iteration (tests)."""
        self._check(load().lobpcg_set_test_faults(self._h, int(mask), int(iteration)), "set_test_faults")

    def set_precond_offset(self, c: float):
        """Diagonal preconditioner shift sigma_j = theta_j - c (theta_max - theta_min); 0 = theta_j."""
        self._check(load().lobpcg_set_precond_offset(self._h, float(c)), "set_precond_offset")
        self.precond_offset = float(c)

    def set_mlp(self, mlp):
        """Attach a network for PRECOND_MLP (None detaches); keep it alive while attached."""
        self._mlp = mlp
        self._check(load().lobpcg_set_mlp(self._h, mlp._h if mlp is not None else None), "set_mlp")

    def features(self, stream=None):
        """(rownorm, tilemean): the per-row network inputs, device float32[n] each."""
        import torch
        r = torch.empty(self.n, dtype=torch.float32, device="cuda")
        t = torch.empty(self.n, dtype=torch.float32, device="cuda")
        self._check(load().lobpcg_get_features(self._h, _dev_ptr(r), _dev_ptr(t), _stream_ptr(stream)), "features")
        return r, t

    def harvest_block(self, X, HX, theta, hb, stream=None):
        """One harvest step on (X, H X, theta) into the HarvestBuffer hb."""
        import torch
        self._check(load().lobpcg_harvest_block(self._h, _dev_ptr(X, self.torch_dtype, "X"),
                                                _dev_ptr(HX, self.torch_dtype, "HX"),
                                                _dev_ptr(theta, torch.float64, "theta"), X.shape[1],
                                                ctypes.byref(hb.h), _stream_ptr(stream)), "harvest_block")
        return hb

    def solve(self, X, nev, tol=1e-6, maxiter=5000, precond=PRECOND_DIAG, history=False, timing=False,
              stream=None, raise_on_noconv=False, harvest=None, raise_on_error=True) -> SolveResult:
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
        if harvest is not None:
            info.harvest = ctypes.cast(ctypes.pointer(harvest.h), ctypes.c_void_p)
        rc = load().lobpcg_solve(self._h, k, nev, _dev_ptr(X, self.torch_dtype, "X"),
                                 evals.ctypes.data_as(ctypes.c_void_p), rel.ctypes.data_as(ctypes.c_void_p),
                                 float(tol), int(maxiter), int(precond), ctypes.byref(info), _stream_ptr(stream))
        if (rc not in (OK, ENOCONV) and raise_on_error) or (rc == ENOCONV and raise_on_noconv):
            self._check(rc, "solve")
        res = SolveResult(evals=evals, rel=rel, status=rc, iters=info.iters, n_spmm=info.n_spmm,
                          p_dropped=info.p_dropped, cholqr_retries=info.cholqr_retries,
                          confirmations=info.confirmations, refreshes=info.refreshes, gamma=info.gamma,
                          cholqr_shifted=info.cholqr_shifted, mlp_fallbacks=info.mlp_fallbacks,
                          locked_max=info.locked_max,
                          times=dict(spmm=info.t_spmm, precond_update=info.t_precond_update, gram=info.t_gram,
                                     rr=info.t_rr, orth=info.t_orth, total=info.t_total))
        if history:
            res.theta_hist = th.reshape(-1, k)[:info.iters]
            res.rel_hist = rh.reshape(-1, k)[:info.iters]
        return res


# -- learned preconditioner ----------------------------------------------------------------------
def pack_params(p: dict) -> np.ndarray:
    """Parameter blob (float32[MLP_NBLOB]) from a dict of arrays named as in MLP_LAYOUT."""
    parts = [np.asarray(p[name], dtype=np.float32).reshape(shape) for name, shape in MLP_LAYOUT]
    blob = np.concatenate([x.ravel() for x in parts]).astype(np.float32)
    assert blob.size == MLP_NBLOB
    return blob


def unpack_params(blob) -> dict:
    blob = np.asarray(blob, dtype=np.float32)
    out, o = {}, 0
    for name, shape in MLP_LAYOUT:
        size = int(np.prod(shape)) if shape else 1
        out[name] = blob[o:o + size].reshape(shape).copy() if shape else float(blob[o])
        o += size
    return out


def _fptr(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_float))


class Mlp:
    """The 4 -> 64 -> 64 -> 1 preconditioner network on the current device."""

    def __init__(self, params):
        lib = load()
        blob = np.ascontiguousarray(params if isinstance(params, np.ndarray) else pack_params(params),
                                    dtype=np.float32)
        h = ctypes.c_void_p()
        rc = lib.lobpcg_mlp_create(ctypes.byref(h), _fptr(blob))
        if rc != OK:
            raise LobpcgError(rc, "mlp_create: " + lib.lobpcg_strerror(rc).decode())
        self._h = h

    def _check(self, rc, what):
        if rc != OK:
            msg = load().lobpcg_mlp_last_error(self._h).decode()
            raise LobpcgError(rc, f"{what}: {msg or load().lobpcg_strerror(rc).decode()}")

    def close(self):
        if getattr(self, "_h", None):
            load().lobpcg_mlp_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_params(self, params):
        blob = np.ascontiguousarray(params if isinstance(params, np.ndarray) else pack_params(params),
                                    dtype=np.float32)
        self._check(load().lobpcg_mlp_set_params(self._h, _fptr(blob)), "set_params")

    def params(self) -> np.ndarray:
        blob = np.zeros(MLP_NBLOB, dtype=np.float32)
        self._check(load().lobpcg_mlp_get_params(self._h, _fptr(blob)), "get_params")
        return blob

    def forward(self, feat, out=None, stream=None):
        import torch
        N = feat.shape[0]
        if out is None:
            out = torch.empty(N, dtype=torch.float32, device=feat.device)
        self._check(load().lobpcg_mlp_forward(self._h, _dev_ptr(feat, torch.float32, "feat"), N,
                                              _dev_ptr(out, torch.float32, "o"), _stream_ptr(stream)), "forward")
        return out

    def fit_standardizer(self, feat, stream=None):
        import torch
        self._check(load().lobpcg_mlp_fit_standardizer(self._h, _dev_ptr(feat, torch.float32, "feat"),
                                                       feat.shape[0], _stream_ptr(stream)), "fit_standardizer")

    def loss_grad(self, batch, stream=None):
        loss = ctypes.c_double()
        g = np.zeros(MLP_NPARAM, dtype=np.float32)
        self._check(load().lobpcg_mlp_loss_grad(self._h, ctypes.byref(batch.b), ctypes.byref(loss), _fptr(g),
                                                _stream_ptr(stream)), "loss_grad")
        return loss.value, g

    def train_step(self, batch, lr, stream=None):
        loss = ctypes.c_double()
        self._check(load().lobpcg_mlp_train_step(self._h, ctypes.byref(batch.b), float(lr), ctypes.byref(loss),
                                                 _stream_ptr(stream)), "train_step")
        return loss.value


class Batch:
    """Device training batch (keeps the tensors alive)."""

    def __init__(self, feat, U, T, w, Xrow, group_off):
        import torch
        self.t = (feat, U, T, w, Xrow, group_off)
        b = MlpBatch()
        b.nsamples = feat.shape[0]
        b.ngroups = group_off.shape[0] - 1
        b.k = Xrow.shape[1]
        b.feat = _dev_ptr(feat, torch.float32, "feat").value
        b.U = _dev_ptr(U, torch.float32, "U").value
        b.T = _dev_ptr(T, torch.float32, "T").value
        b.w = _dev_ptr(w, torch.float32, "w").value
        b.Xrow = _dev_ptr(Xrow, torch.float32, "Xrow").value
        b.group_off = _dev_ptr(group_off, torch.int64, "group_off").value
        self.b = b


class HarvestBuffer:
    """Device arrays a solve (or harvest_block) appends training samples to."""

    def __init__(self, capacity, capacity_groups, k, xstar, nev, every=1, rows=1024, seed=0, rows_index=True):
        import torch
        dev = xstar.device
        self.feat = torch.zeros((capacity, 4), dtype=torch.float32, device=dev)
        self.U = torch.zeros(capacity, dtype=torch.float32, device=dev)
        self.T = torch.zeros(capacity, dtype=torch.float32, device=dev)
        self.w = torch.zeros(capacity, dtype=torch.float32, device=dev)
        self.Xrow = torch.zeros((capacity, k), dtype=torch.float32, device=dev)
        self.row = torch.zeros(capacity, dtype=torch.int32, device=dev) if rows_index else None
        self.group_off = torch.zeros(capacity_groups + 1, dtype=torch.int64, device=dev)
        self.k = k
        h = Harvest()
        h.every, h.rows, h.nev, h.seed = every, rows, nev, seed
        h.capacity, h.capacity_groups = capacity, capacity_groups
        h.feat, h.U, h.T, h.w = (self.feat.data_ptr(), self.U.data_ptr(), self.T.data_ptr(), self.w.data_ptr())
        h.Xrow = self.Xrow.data_ptr()
        h.row = self.row.data_ptr() if self.row is not None else None
        h.group_off = self.group_off.data_ptr()
        self.h = h
        self.set_xstar(xstar, nev)

    def set_xstar(self, xstar, nev=None, seed=None):
        if not xstar.is_contiguous():
            raise ValueError("xstar must be contiguous")
        self._xstar = xstar
        self.h.xstar = xstar.data_ptr()
        if nev is not None:
            self.h.nev = nev
        if seed is not None:
            self.h.seed = seed

    @property
    def nsamples(self):
        return int(self.h.nsamples)

    @property
    def ngroups(self):
        return int(self.h.ngroups)

    @property
    def full(self):
        return bool(self.h.full)

    def batch(self):
        n, g = self.nsamples, self.ngroups
        return Batch(self.feat[:n], self.U[:n], self.T[:n], self.w[:n], self.Xrow[:n], self.group_off[:g + 1])
