"""Python binding of libtls (ctypes over the C ABI declared in include/tls.h).

Argument marshalling only: every step of the computation runs in the HIP
kernels of libtls. PyTorch provides device memory (workspaces, vectors)
and the current HIP stream. The binding fails loudly when the library is
not built; there is no CPU fallback.

The functions keep the C names:

    P, rep = tls_factor_precond(A, u_q="fp64", scaling=True)
    omega, trace = tls_pcg_step(P, sigma2, rhs, l, u_p="fp64", trace=True)
    x, sigma, stats = tls_rqi_solve(A, b, P, opts)

``A`` is a :class:`Matrix` (see :func:`dense` and :func:`csr`).
"""
from __future__ import annotations

import ctypes as C
import dataclasses
import math
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "lib", "libtls.so")

PREC = {"fp64": 0, "fp32": 1, "fp16": 2, "bf16": 3, "bf16x3": 4}
PREC_NAME = {v: k for k, v in PREC.items()}
DENSE, CSR_FMT = 0, 1
MAX_ITERS = 256

STATUS = {
    0: "TLS_OK", -1: "TLS_ERR_ARG", -2: "TLS_ERR_HIP", -3: "TLS_ERR_NOT_SPD",
    -4: "TLS_ERR_PRECISION", -5: "TLS_ERR_INDEFINITE", -6: "TLS_ERR_NONUNIQUE",
    -7: "TLS_ERR_NO_CONVERGENCE", -8: "TLS_ERR_WORKSPACE", -9: "TLS_ERR_NONFINITE",
    -10: "TLS_ERR_SYNC_TIMEOUT",
}


class TLSError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


# ----------------------------------------------------------------------------
# C structures (must match include/tls.h)
# ----------------------------------------------------------------------------
class c_matrix(C.Structure):
    _fields_ = [("format", C.c_int32), ("reserved", C.c_int32), ("m", C.c_int64),
                ("n", C.c_int64), ("ld", C.c_int64), ("nnz", C.c_int64),
                ("val", C.c_void_p), ("row_ptr", C.c_void_p), ("col_idx", C.c_void_p)]


class c_gate_report(C.Structure):
    _fields_ = [(k, C.c_double) for k in (
        "kappa_est", "kappaF_est", "sigma_n_est", "sigma_1_est", "lam_min_H", "bound5",
        "bound_chol", "bound_wilkinson", "bound_hp", "bound6", "u_q", "ctilde_min",
        "quality_lo", "quality_hi", "cert_margin")] + \
        [(k, C.c_int32) for k in ("requested", "used", "verdict", "escalations",
                                  "chol_retries", "lanczos_steps", "method", "reserved")]

    def to_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


MLP_IN = 32
MLP_WIDTH = 256
MLP_PARAMS = 140289


class c_rqi_opts(C.Structure):
    _fields_ = [(k, C.c_int32) for k in (
        "u_p", "kmax", "stop_patience", "stop_ge", "ls_corrections", "strict_pd",
        "shift_clamp", "refine_sweeps", "refine_pcg_steps", "allow_escalate",
        "gate_enforce", "features", "min_inner_steps", "step_margin")] + \
        [("shift_clamp_tau", C.c_double), ("sigma0_hint", C.c_double), ("psi_tie", C.c_double),
         ("x_snapshots", C.c_void_p), ("mlp_theta", C.c_void_p), ("mlp_norm", C.c_void_p)]


_OPT_FIELDS = {name for name, _ in c_rqi_opts._fields_}


class c_rqi_stats(C.Structure):
    _fields_ = [(k, C.c_int32) for k in (
        "iters", "k_best", "pcg_steps", "warm_used", "stopped", "negative_delta",
        "refine_steps", "clamped", "gate_async", "ls_refined")] + \
        [("sigma_ls", C.c_double), ("psi", C.c_double * MAX_ITERS),
         ("sigma", C.c_double * MAX_ITERS), ("t_ms", C.c_double * MAX_ITERS),
         ("t_factor_ms", C.c_double), ("t_total_ms", C.c_double), ("sigma_final", C.c_double),
         ("sigma_hat", C.c_double), ("psi_warm", C.c_double), ("psi_plain", C.c_double),
         ("t_verdict_ms", C.c_double), ("features", C.c_float * MLP_IN)]

    def to_dict(self):
        k = self.iters
        return {
            "iters": k, "k_best": self.k_best, "pcg_steps": self.pcg_steps,
            "warm_used": self.warm_used, "stopped": self.stopped,
            "negative_delta": self.negative_delta, "refine_steps": self.refine_steps,
            "clamped": self.clamped, "gate_async": self.gate_async, "ls_refined": self.ls_refined,
            "sigma_ls": self.sigma_ls,
            "psi": list(self.psi[:k]), "sigma": list(self.sigma[:k]), "t_ms": list(self.t_ms[:k]),
            "t_factor_ms": self.t_factor_ms, "t_total_ms": self.t_total_ms,
            "sigma_final": self.sigma_final, "sigma_hat": self.sigma_hat,
            "psi_warm": self.psi_warm, "psi_plain": self.psi_plain,
            "t_verdict_ms": self.t_verdict_ms, "features": list(self.features),
        }


PROF_CLASSES = ["precond_apply", "pcg_step", "gram", "chol_panel", "chol_update", "residual",
                "gradient", "outer_scalars", "setup", "lanczos", "pack", "residual_dd", "invert",
                "mlp", "gate", "qr"]


class c_kernel_times(C.Structure):
    _fields_ = [("launches", C.c_int32 * len(PROF_CLASSES)),
                ("total_ms", C.c_double * len(PROF_CLASSES))]


# ----------------------------------------------------------------------------
# library loading
# ----------------------------------------------------------------------------
_lib = None

_SIGS = {
    "tls_last_error": (C.c_char_p, []),
    "tls_version": (C.c_char_p, []),
    "tls_default_opts": (None, [C.POINTER(c_rqi_opts)]),
    "tls_factor_workspace_size": (C.c_size_t, [C.POINTER(c_matrix), C.c_int32]),
    "tls_factor_precond": (C.c_int, [C.POINTER(c_matrix), C.c_int32, C.c_int32, C.c_int32,
                                     C.c_void_p, C.c_size_t, C.c_void_p, C.POINTER(C.c_void_p),
                                     C.POINTER(c_gate_report)]),
    "tls_gram": (C.c_int, [C.POINTER(c_matrix), C.c_int32, C.c_int32, C.c_void_p, C.c_void_p,
                           C.c_void_p, C.c_size_t, C.c_void_p]),
    "tls_factor_qr_workspace_size": (C.c_size_t, [C.POINTER(c_matrix), C.c_int32]),
    "tls_factor_precond_qr": (C.c_int, [C.POINTER(c_matrix), C.c_int32, C.c_int32, C.c_int32,
                                        C.c_void_p, C.c_size_t, C.c_void_p, C.POINTER(C.c_void_p),
                                        C.POINTER(c_gate_report)]),
    "tls_precond_import_workspace_size": (C.c_size_t, [C.c_int64]),
    "tls_precond_import": (C.c_int, [C.c_int64, C.c_void_p, C.c_void_p, C.c_int32, C.c_void_p,
                                     C.c_size_t, C.c_void_p, C.POINTER(C.c_void_p)]),
    "tls_precond_destroy": (None, [C.c_void_p]),
    "tls_precond_info": (C.c_int, [C.c_void_p, C.POINTER(C.c_int64), C.POINTER(C.c_int32),
                                   C.POINTER(c_gate_report)]),
    "tls_precond_export": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "tls_pcg_workspace_size": (C.c_size_t, [C.c_void_p, C.c_int32, C.c_int32]),
    "tls_pcg_step": (C.c_int, [C.c_void_p, C.c_double, C.c_int32, C.c_void_p, C.c_void_p,
                               C.c_int32, C.c_int32, C.c_int32, C.c_void_p, C.c_size_t,
                               C.c_void_p, C.c_void_p]),
    "tls_pcg_step_noalloc": (C.c_int, [C.c_void_p, C.c_double, C.c_int32, C.c_void_p,
                                       C.c_void_p, C.c_int32, C.c_int32, C.c_int32, C.c_void_p,
                                       C.c_void_p]),
    "tls_apply_precond": (C.c_int, [C.c_void_p, C.c_int32, C.c_int32, C.c_void_p, C.c_void_p,
                                    C.c_int32, C.c_void_p, C.c_size_t, C.c_void_p]),
    "tls_matvec": (C.c_int, [C.POINTER(c_matrix), C.c_void_p, C.c_int32, C.c_void_p,
                             C.c_void_p, C.c_void_p]),
    "tls_rqi_workspace_size": (C.c_size_t, [C.POINTER(c_matrix), C.c_void_p,
                                            C.POINTER(c_rqi_opts)]),
    "tls_rqi_solve": (C.c_int, [C.POINTER(c_matrix), C.c_void_p, C.c_void_p,
                                C.POINTER(c_rqi_opts), C.c_void_p, C.POINTER(C.c_double),
                                C.POINTER(c_rqi_stats), C.c_void_p, C.c_size_t, C.c_void_p]),
    "tls_round": (C.c_int, [C.c_void_p, C.c_int64, C.c_int32, C.c_void_p, C.c_void_p]),
    "tls_mlp_workspace_size": (C.c_size_t, [C.c_int64]),
    "tls_mlp_forward": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64, C.c_void_p,
                                  C.c_void_p, C.c_size_t, C.c_void_p]),
    "tls_mlp_loss_grad": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64,
                                    C.c_void_p, C.c_void_p, C.c_void_p, C.c_size_t, C.c_void_p]),
    "tls_mlp_adam": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64,
                               C.c_int64, C.c_float, C.c_float, C.c_float, C.c_float,
                               C.c_void_p]),
    "tls_profile_start": (C.c_int, []),
    "tls_precond_set_apply": (C.c_int, [C.c_void_p, C.c_int32]),
    "tls_profile_stop": (C.c_int, [C.POINTER(c_kernel_times)]),
}


def lib():
    """Load libtls.so (raises when it is not built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"libtls.so is not built ({LIB_PATH}); run __graft_entry__.build()")
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def _check(status: int):
    if status != 0:
        raise TLSError(status, lib().tls_last_error().decode())


def _torch():
    import torch
    if not torch.cuda.is_available():
        raise RuntimeError("no GPU visible: libtls runs on MI355X only")
    return torch


def _stream():
    torch = _torch()
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t) -> C.c_void_p:
    return C.c_void_p(t.data_ptr()) if t is not None else C.c_void_p(0)


class Workspace:
    """A 256-byte aligned device buffer carved from a torch uint8 tensor."""

    def __init__(self, nbytes: int, device="cuda"):
        torch = _torch()
        self.nbytes = int(nbytes)
        self._buf = torch.empty(self.nbytes + 256, dtype=torch.uint8, device=device)
        base = self._buf.data_ptr()
        self.off = (-base) % 256
        self.ptr = C.c_void_p(base + self.off)


# ----------------------------------------------------------------------------
# matrices
# ----------------------------------------------------------------------------
@dataclasses.dataclass
class Matrix:
    c: c_matrix
    tensors: tuple     # keep device arrays alive
    m: int
    n: int
    fmt: int


def dense(A, device="cuda") -> Matrix:
    """Column-major FP64 device copy of a dense m x n array (numpy or torch)."""
    torch = _torch()
    if isinstance(A, np.ndarray):
        At = torch.from_numpy(np.asfortranarray(A, dtype=np.float64).T.copy()).to(device)
    else:
        At = A.to(device=device, dtype=torch.float64).t().contiguous()
    n, m = At.shape                  # At is A^T row-major == A column-major
    c = c_matrix(DENSE, 0, m, n, m, 0, At.data_ptr(), None, None)
    return Matrix(c, (At,), m, n, DENSE)


def dense_t(At, m=None) -> Matrix:
    """A dense m x n matrix given as its transpose At (an n x ld row-major
    float64 device tensor, i.e. A column-major with leading dimension ld);
    m (default ld) rows of each column are A's, the rest padding; no copy."""
    torch = _torch()
    if not (isinstance(At, torch.Tensor) and At.is_cuda and At.dtype == torch.float64 and At.is_contiguous()):
        raise TypeError("dense_t needs a contiguous float64 device tensor")
    n, ld = At.shape
    m = ld if m is None else int(m)
    if not 0 < m <= ld:
        raise ValueError("need 0 < m <= ld")
    c = c_matrix(DENSE, 0, m, n, ld, 0, At.data_ptr(), None, None)
    return Matrix(c, (At,), m, n, DENSE)


def csr(row_ptr, col_idx, val, m, n, device="cuda") -> Matrix:
    """CSR m x n with int32 indices and float64 values (numpy arrays or
    torch tensors; device tensors of the right types are used in place)."""
    torch = _torch()

    def dev(v, npdt, tdt):
        if isinstance(v, torch.Tensor):
            return v.to(device=device, dtype=tdt).contiguous()
        return torch.as_tensor(np.asarray(v, dtype=npdt)).to(device)
    rp = dev(row_ptr, np.int32, torch.int32)
    ci = dev(col_idx, np.int32, torch.int32)
    va = dev(val, np.float64, torch.float64)
    c = c_matrix(CSR_FMT, 0, m, n, 0, int(ci.numel()), va.data_ptr(), rp.data_ptr(), ci.data_ptr())
    return Matrix(c, (rp, ci, va), m, n, CSR_FMT)


def from_tlsgen(A) -> Matrix:
    """Device copy of a tlsgen output (CSR dataclass or dense array)."""
    if hasattr(A, "row_ptr"):
        return csr(A.row_ptr, A.col_idx, A.val, A.m, A.n)
    return dense(A)


def device_vector(v, device="cuda"):
    torch = _torch()
    return torch.as_tensor(np.ascontiguousarray(v, dtype=np.float64)).to(device)


# ----------------------------------------------------------------------------
# preconditioner
# ----------------------------------------------------------------------------
class Precond:
    def __init__(self, handle, ws, A=None):
        self.handle = handle
        self.ws = ws
        self.A = A

    def __del__(self):
        try:
            if self.handle and _lib is not None:
                _lib.tls_precond_destroy(self.handle)
        except Exception:
            pass
        self.handle = None

    @property
    def n(self) -> int:
        n = C.c_int64()
        st = C.c_int32()
        _check(lib().tls_precond_info(self.handle, C.byref(n), C.byref(st), None))
        return n.value

    def set_apply(self, mode):
        """0: explicit-inverse GEMV split over the chip (default);
        1: blocked substitution; 2: explicit-inverse GEMV, one workgroup per block row."""
        m = {"inverse": 0, "substitution": 1, "inverse_rows": 2}.get(mode, mode)
        _check(lib().tls_precond_set_apply(self.handle, int(m)))

    def info(self):
        n = C.c_int64()
        st = C.c_int32()
        rep = c_gate_report()
        _check(lib().tls_precond_info(self.handle, C.byref(n), C.byref(st), C.byref(rep)))
        return {"n": n.value, "storage": PREC_NAME[st.value], "gate": rep.to_dict()}


def _prec(p) -> int:
    return PREC[p] if isinstance(p, str) else int(p)


def _factor(size_fn, call_fn, A, u_q, scaling, allow_escalate, wait_gate):
    nb = size_fn(C.byref(A.c), _prec(u_q))
    if nb == 0:
        _check(-1)
    ws = Workspace(nb)
    h = C.c_void_p()
    rep = c_gate_report()
    _check(call_fn(C.byref(A.c), _prec(u_q), int(scaling), int(allow_escalate),
                   ws.ptr, ws.nbytes, _stream(), C.byref(h),
                   C.byref(rep) if wait_gate else None))
    return Precond(h, ws, A), (rep.to_dict() if wait_gate else None)


def tls_factor_precond(A: Matrix, u_q="fp64", scaling=True, allow_escalate=False, wait_gate=True):
    """Build the preconditioner of A (see tls.h). Returns (Precond, gate report
    dict). With wait_gate=False the gate's Lanczos runs of a low-precision
    factor finish in the background (the solve overlaps them) and the report
    is None; Precond.info() waits for them."""
    L = lib()
    return _factor(L.tls_factor_workspace_size, L.tls_factor_precond, A, u_q, scaling,
                   allow_escalate, wait_gate)


def tls_gram(A: Matrix, u_q="fp64", scaling=True):
    """The Gram matrix the factorization forms (see tls.h): returns (G upper
    triangle as an n x n float64 tensor, lower part zero; d)."""
    torch = _torch()
    L = lib()
    nb = L.tls_factor_workspace_size(C.byref(A.c), _prec(u_q))
    if nb == 0:
        _check(-1)
    ws = Workspace(nb)
    G = torch.zeros((A.n, A.n), dtype=torch.float64, device="cuda")   # column-major = G^T row-major
    d = torch.empty(A.n, dtype=torch.float64, device="cuda")
    _check(L.tls_gram(C.byref(A.c), _prec(u_q), int(bool(scaling)), _ptr(G), _ptr(d), ws.ptr, ws.nbytes,
                      _stream()))
    return G.t(), d


def tls_factor_precond_qr(A: Matrix, u_q="fp64", scaling=True, allow_escalate=False, wait_gate=True):
    """The preconditioner from the Householder QR of A (see tls.h); same
    returns and options as tls_factor_precond."""
    L = lib()
    return _factor(L.tls_factor_qr_workspace_size, L.tls_factor_precond_qr, A, u_q, scaling,
                   allow_escalate, wait_gate)


def tls_precond_import(R, d=None, storage="fp64"):
    """Wrap a host factor R (n x n upper) and scaling d (R = R_hat diag(d))."""
    L = lib()
    R = np.asfortranarray(R, dtype=np.float64)
    n = R.shape[0]
    nb = L.tls_precond_import_workspace_size(n)
    ws = Workspace(nb)
    h = C.c_void_p()
    dd = None if d is None else np.ascontiguousarray(d, dtype=np.float64)
    _check(L.tls_precond_import(n, R.ctypes.data_as(C.c_void_p),
                                None if dd is None else dd.ctypes.data_as(C.c_void_p),
                                _prec(storage), ws.ptr, ws.nbytes, _stream(), C.byref(h)))
    P = Precond(h, ws)
    P._keep = (R, dd)
    return P


def tls_precond_export(P: Precond):
    """(R_hat, d) on the host as float64 arrays."""
    n = P.n
    R = np.zeros((n, n), order="F")
    d = np.zeros(n)
    _check(lib().tls_precond_export(P.handle, R.ctypes.data_as(C.c_void_p),
                                    d.ctypes.data_as(C.c_void_p), _stream()))
    return R, d


# ----------------------------------------------------------------------------
# solves
# ----------------------------------------------------------------------------
def _as_cols(v, n):
    torch = _torch()
    t = torch.as_tensor(v) if not hasattr(v, "data_ptr") else v
    t = t.to(device="cuda", dtype=torch.float64)
    if t.dim() == 1:
        t = t.reshape(1, n)
    elif t.shape[0] == n and t.dim() == 2 and t.shape[1] in (1, 2) and t.shape[0] != t.shape[1]:
        t = t.t()
    return t.contiguous()     # [nrhs][n]: columns stored one after another


def tls_pcg_step(P: Precond, sigma2: float, rhs, l: int, u_p="fp64", strict=False,
                 trace=False):
    """Algorithm 3 on nrhs = 1 or 2 right-hand sides (rows of a [nrhs, n]
    tensor or a length-n vector). Returns (omega [nrhs, n], trace dict or None)."""
    torch = _torch()
    n = P.n
    R = _as_cols(rhs, n)
    nrhs = R.shape[0]
    out = torch.empty_like(R)
    L = lib()
    nb = L.tls_pcg_workspace_size(P.handle, nrhs, l)
    ws = Workspace(nb)
    tr = np.full(nrhs * 4 * (l + 2), np.nan) if trace else None
    _check(L.tls_pcg_step(P.handle, float(sigma2), nrhs, _ptr(R), _ptr(out), int(l), _prec(u_p),
                          int(strict), ws.ptr, ws.nbytes, _stream(),
                          tr.ctypes.data_as(C.c_void_p) if trace else None))
    tdict = None
    if trace:
        tr = tr.reshape(nrhs, 4, l + 2)
        tdict = {"eta": tr[:, 0], "delta": tr[:, 1], "alpha": tr[:, 2], "beta": tr[:, 3]}
    return out, tdict


def tls_pcg_step_noalloc(P: Precond, sigma2: float, rhs, l: int, u_p="fp64", strict=False,
                         trace=False):
    """tls_pcg_step with the library's static scratch in place of a workspace
    (no device allocation inside the call). Returns (omega, trace dict or None)."""
    n = P.n
    R = _as_cols(rhs, n)
    nrhs = R.shape[0]
    out = _torch().empty_like(R)
    tr = np.full(nrhs * 4 * (l + 2), np.nan) if trace else None
    _check(lib().tls_pcg_step_noalloc(P.handle, float(sigma2), nrhs, _ptr(R), _ptr(out), int(l),
                                      _prec(u_p), int(strict), _stream(),
                                      tr.ctypes.data_as(C.c_void_p) if trace else None))
    tdict = None
    if trace:
        tr = tr.reshape(nrhs, 4, l + 2)
        tdict = {"eta": tr[:, 0], "delta": tr[:, 1], "alpha": tr[:, 2], "beta": tr[:, 3]}
    return out, tdict


def tls_apply_precond(P: Precond, trans: int, v, u_p="fp64"):
    """R^{-1} v (trans = 0) or R^{-T} v (trans = 1)."""
    torch = _torch()
    n = P.n
    V = _as_cols(v, n)
    out = torch.empty_like(V)
    L = lib()
    ws = Workspace(L.tls_pcg_workspace_size(P.handle, V.shape[0], 0))
    _check(L.tls_apply_precond(P.handle, int(trans), V.shape[0], _ptr(V), _ptr(out), _prec(u_p),
                               ws.ptr, ws.nbytes, _stream()))
    return out


def tls_matvec(A: Matrix, P, trans: int, x):
    torch = _torch()
    xt = torch.as_tensor(x).to(device="cuda", dtype=torch.float64).contiguous()
    y = torch.empty(A.n if trans else A.m, dtype=torch.float64, device="cuda")
    _check(lib().tls_matvec(C.byref(A.c), P.handle if P is not None else None, int(trans),
                            _ptr(xt), _ptr(y), _stream()))
    return y


def tls_round(v, prec):
    """Round FP64 values to `prec` (round to nearest even), returned as FP64."""
    torch = _torch()
    t = torch.as_tensor(np.ascontiguousarray(v, dtype=np.float64)).to("cuda")
    out = torch.empty_like(t)
    _check(lib().tls_round(_ptr(t), t.numel(), _prec(prec), _ptr(out), _stream()))
    return out


def default_opts(**kw) -> c_rqi_opts:
    o = c_rqi_opts()
    lib().tls_default_opts(C.byref(o))
    for k, v in kw.items():
        if k == "u_p":
            v = _prec(v)
        if k == "x_snapshots":
            v = v.data_ptr() if v is not None else None
        if k == "mlp":
            # (theta, norm) device float32 tensors; the caller keeps them alive
            theta, norm = v if v is not None else (None, None)
            o.mlp_theta = theta.data_ptr() if theta is not None else None
            o.mlp_norm = norm.data_ptr() if norm is not None else None
            continue
        if k not in _OPT_FIELDS:
            raise TypeError(f"unknown option {k!r}")
        setattr(o, k, v)
    return o


def tls_rqi_solve(A: Matrix, b, P: Precond, opts: c_rqi_opts | None = None, x_out=None,
                  allow_no_convergence=False):
    """Algorithm 2 / 4. Returns (x [n] device tensor, sigma, stats dict)."""
    torch = _torch()
    if opts is None:
        opts = default_opts()
    bt = torch.as_tensor(b).to(device="cuda", dtype=torch.float64).contiguous()
    x = x_out if x_out is not None else torch.empty(A.n, dtype=torch.float64, device="cuda")
    L = lib()
    nb = L.tls_rqi_workspace_size(C.byref(A.c), P.handle, C.byref(opts))
    if nb == 0:
        raise TLSError(-1, "tls_rqi_workspace_size returned 0")
    ws = Workspace(nb)
    sig = C.c_double()
    st = c_rqi_stats()
    status = L.tls_rqi_solve(C.byref(A.c), _ptr(bt), P.handle, C.byref(opts), _ptr(x),
                             C.byref(sig), C.byref(st), ws.ptr, ws.nbytes, _stream())
    if status != 0 and not (allow_no_convergence and status == -7):
        _check(status)
    d = st.to_dict()
    d["status"] = STATUS.get(status, status)
    return x, sig.value, d


def tls_profile_start():
    _check(lib().tls_profile_start())


def tls_profile_stop():
    """Per kernel class: {name: (launches, total_ms)} since tls_profile_start."""
    t = c_kernel_times()
    _check(lib().tls_profile_stop(C.byref(t)))
    return {name: (t.launches[i], t.total_ms[i]) for i, name in enumerate(PROF_CLASSES)}


# ----------------------------------------------------------------------------
# warm-start network
# ----------------------------------------------------------------------------
def _f32(t):
    torch = _torch()
    return torch.as_tensor(t).to(device="cuda", dtype=torch.float32).contiguous()


def tls_mlp_forward(theta, norm, X):
    """y (batch,) = network(X) on the device (float32 tensors)."""
    torch = _torch()
    th, nm, Xd = _f32(theta), _f32(norm), _f32(X)
    B = Xd.shape[0]
    y = torch.empty(B, dtype=torch.float32, device="cuda")
    ws = Workspace(lib().tls_mlp_workspace_size(B))
    _check(lib().tls_mlp_forward(_ptr(th), _ptr(nm), _ptr(Xd), B, _ptr(y), ws.ptr, ws.nbytes,
                                 _stream()))
    return y


def tls_mlp_loss_grad(theta, norm, X, t, grad_out=None, ws=None):
    """(loss [1] device tensor, grad [MLP_PARAMS] device tensor)."""
    torch = _torch()
    th, nm, Xd, td = _f32(theta), _f32(norm), _f32(X), _f32(t)
    B = Xd.shape[0]
    g = grad_out if grad_out is not None else torch.empty(MLP_PARAMS, dtype=torch.float32, device="cuda")
    loss = torch.empty(1, dtype=torch.float32, device="cuda")
    need = lib().tls_mlp_workspace_size(B)
    if ws is None or ws.nbytes < need:
        ws = Workspace(need)
    _check(lib().tls_mlp_loss_grad(_ptr(th), _ptr(nm), _ptr(Xd), _ptr(td), B, _ptr(g), _ptr(loss),
                                   ws.ptr, ws.nbytes, _stream()))
    return loss, g


def tls_mlp_adam(theta, m, v, grad, step, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """In-place Adam update of the float32 device tensors theta, m, v."""
    _check(lib().tls_mlp_adam(_ptr(theta), _ptr(m), _ptr(v), _ptr(grad), theta.numel(), step,
                              lr, beta1, beta2, eps, _stream()))
