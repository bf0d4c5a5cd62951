"""Band-Lanczos block MINRES on AMD Instinct MI355X (gfx950).

Thin Python binding of libbmr.so (C ABI in include/bmr.h): argument
marshalling only.  Every step of the solve runs in the library's HIP
kernels; PyTorch provides device memory and the current stream.  There is no
CPU fallback: without the built library every call raises.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass, field
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libbmr.so")

MAX_P = 16
MAX_BENCH = 4


def group_len(p: int) -> int:
    """Blocks per group of search directions (the library applies eq. (4.2)
    once per group): min(32, 2048 // p^2) for p <= 8, max(2, 1024 // p^2)
    above, as in the library."""
    return min(32, 2048 // (p * p)) if p <= 8 else max(2, 1024 // (p * p))

CONVERGED = 0
MAX_ITER = 1
BENCH_EXHAUSTED = 2
STAGNATED = 3
INVALID_ARG = -1
WORKSPACE_TOO_SMALL = -2
HIP_ERROR = -3
NONFINITE = -4
SINGULAR_R = -5
IC0_BREAKDOWN = -6


class _Csr(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("nnz", ctypes.c_int64), ("row_ptr", ctypes.c_void_p),
                ("col_idx", ctypes.c_void_p), ("val", ctypes.c_void_p)]


class _Opts(ctypes.Structure):
    _fields_ = [("tol", ctypes.c_double), ("max_iter", ctypes.c_int64), ("gamma", ctypes.c_double),
                ("n_bench", ctypes.c_int32), ("poll_every", ctypes.c_int32), ("seed", ctypes.c_uint64),
                ("hist_cap", ctypes.c_int64), ("flags", ctypes.c_uint32), ("precision", ctypes.c_int32),
                ("inner_tol", ctypes.c_double), ("max_refine", ctypes.c_int32), ("precond", ctypes.c_int32),
                ("relax_tol", ctypes.c_double)]


class _Stats(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("n_replaced", ctypes.c_int32), ("band_iters", ctypes.c_int64),
                ("block_iters", ctypes.c_int64), ("n_explicit_qr", ctypes.c_int32), ("p", ctypes.c_int32),
                ("res_rec", ctypes.c_double * MAX_P), ("time_ms", ctypes.c_double),
                ("t_kernel_ms", ctypes.c_double * 4), ("n_profiled", ctypes.c_int64),
                ("precision", ctypes.c_int32), ("n_refine", ctypes.c_int32), ("res_true", ctypes.c_double * MAX_P),
                ("res_explicit", ctypes.c_double * MAX_P), ("n_retained", ctypes.c_int32), ("_pad", ctypes.c_int32),
                ("switch_iter", ctypes.c_int64)]

FLAG_PROFILE = 1
FLAG_RETAIN = 2
FLAG_ACCUMULATE = 4
PREC_FP64 = 0
PREC_MIXED = 1
PREC_RELAXED = 2
_PRECISIONS = {"fp64": PREC_FP64, "mixed": PREC_MIXED, "relaxed": PREC_RELAXED}
KERNEL_NAMES = ("pass1_spmm_gram", "reduce", "band", "pass2_update")


PRECOND_NONE = 0
PRECOND_IC0 = 1
_PRECONDS = {"none": PRECOND_NONE, "ic0": PRECOND_IC0}

EXPORTS = ("bmr_version", "bmr_status_string", "bmr_default_opts", "bmr_workspace_bytes", "bmr_solve",
           "bmr_spmm", "bmr_spmm_f32", "bmr_pattern_grad", "bmr_residual", "bmr_residual_noalloc", "bmr_ic0_bytes", "bmr_ic0_factor",
           "bmr_ic0_apply", "bmr_solve_ic0")

_lib = None


def load(path: str = LIB_PATH):
    """Load libbmr.so (once).  Raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"libbmr.so not found at {path}; run `python -m paper_1301_2102_amd.build`")
    lib = ctypes.CDLL(path)
    vp, i32, i64, sz = ctypes.c_void_p, ctypes.c_int, ctypes.c_int64, ctypes.c_size_t
    lib.bmr_version.restype = i32
    lib.bmr_version.argtypes = []
    lib.bmr_status_string.restype = ctypes.c_char_p
    lib.bmr_status_string.argtypes = [i32]
    lib.bmr_default_opts.restype = None
    lib.bmr_default_opts.argtypes = [ctypes.POINTER(_Opts)]
    lib.bmr_workspace_bytes.restype = i32
    lib.bmr_workspace_bytes.argtypes = [i64, i64, i32, ctypes.POINTER(_Opts), ctypes.POINTER(sz)]
    lib.bmr_solve.restype = i32
    lib.bmr_solve.argtypes = [ctypes.POINTER(_Csr), vp, vp, i32, ctypes.POINTER(_Opts), vp, sz, vp,
                              ctypes.POINTER(_Stats), vp]
    lib.bmr_spmm.restype = i32
    lib.bmr_spmm.argtypes = [ctypes.POINTER(_Csr), vp, vp, i32, vp]
    lib.bmr_spmm_f32.restype = i32
    lib.bmr_spmm_f32.argtypes = [ctypes.POINTER(_Csr), vp, vp, vp, i32, vp]
    lib.bmr_pattern_grad.restype = i32
    lib.bmr_pattern_grad.argtypes = [ctypes.POINTER(_Csr), vp, vp, i32, vp, vp]
    lib.bmr_residual.restype = i32
    lib.bmr_residual.argtypes = [ctypes.POINTER(_Csr), vp, vp, i32, vp, ctypes.POINTER(ctypes.c_double), vp, sz, vp]
    lib.bmr_ic0_bytes.restype = i32
    lib.bmr_ic0_bytes.argtypes = [i64, i64, ctypes.POINTER(sz)]
    lib.bmr_ic0_factor.restype = i32
    lib.bmr_ic0_factor.argtypes = [ctypes.POINTER(_Csr), vp, sz, vp]
    lib.bmr_ic0_apply.restype = i32
    lib.bmr_ic0_apply.argtypes = [vp, vp, vp, i32, i32, vp]
    lib.bmr_solve_ic0.restype = i32
    lib.bmr_solve_ic0.argtypes = [ctypes.POINTER(_Csr), vp, vp, vp, i32, ctypes.POINTER(_Opts), vp, sz, vp,
                                  ctypes.POINTER(_Stats), vp]
    _lib = lib
    return lib


def status_string(status: int) -> str:
    return load().bmr_status_string(int(status)).decode()


class BmrError(RuntimeError):
    def __init__(self, status: int, what: str):
        super().__init__(f"{what}: {status_string(status)} ({status})")
        self.status = status


# ---------------------------------------------------------------------------
# device-side matrix
# ---------------------------------------------------------------------------
@dataclass
class DeviceCsr:
    """CSR arrays resident on a GPU (torch tensors: int32, int32, float64)."""
    n: int
    row_ptr: "object"
    col_idx: "object"
    val: "object"

    @property
    def nnz(self) -> int:
        return int(self.col_idx.numel())

    def _c(self) -> _Csr:
        return _Csr(self.n, self.nnz, self.row_ptr.data_ptr(), self.col_idx.data_ptr(), self.val.data_ptr())


def to_device(A, device="cuda") -> DeviceCsr:
    """Copy a host CSR (anything with n/indptr/indices/data) to the device."""
    import torch
    return DeviceCsr(int(A.n),
                     torch.from_numpy(np.ascontiguousarray(A.indptr, dtype=np.int32)).to(device),
                     torch.from_numpy(np.ascontiguousarray(A.indices, dtype=np.int32)).to(device),
                     torch.from_numpy(np.ascontiguousarray(A.data, dtype=np.float64)).to(device))


def _stream_handle(device):
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def _check_block(t, n, name, dtype=None):
    import torch
    dtype = torch.float64 if dtype is None else dtype
    if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == dtype and t.dim() == 2
            and t.shape[0] == n and t.is_contiguous()):
        raise ValueError(f"{name} must be a contiguous {dtype} CUDA tensor of shape (n, p)")


def _opts(tol, max_iter, gamma, n_bench, seed, hist_cap, poll_every, flags=0, precision="fp64", inner_tol=None,
          max_refine=None, relax_tol=None) -> _Opts:
    o = _Opts()
    load().bmr_default_opts(ctypes.byref(o))
    o.tol, o.max_iter, o.gamma, o.n_bench = float(tol), int(max_iter), float(gamma), int(n_bench)
    o.seed, o.hist_cap, o.poll_every = int(seed) & 0xFFFFFFFFFFFFFFFF, int(hist_cap), int(poll_every)
    o.flags = int(flags)
    if precision not in _PRECISIONS:
        raise ValueError(f"precision must be one of {sorted(_PRECISIONS)}")
    o.precision = _PRECISIONS[precision]
    if inner_tol is not None:
        o.inner_tol = float(inner_tol)
    if max_refine is not None:
        o.max_refine = int(max_refine)
    if relax_tol is not None:
        o.relax_tol = float(relax_tol)
    return o


def workspace_bytes(n: int, p: int, n_bench: int = 2, hist_cap: int = 0, nnz: int = 0,
                    precision: str = "fp64", precond: str = "none", retain: bool = False) -> int:
    """Device workspace bytes of a solve (nnz matters for precision="mixed" and "relaxed";
    precond="ic0" for a preconditioned solve; retain for kept candidates)."""
    o = _opts(1e-8, 1, 1e-10, n_bench, 0, hist_cap, 0, flags=FLAG_RETAIN if retain else 0, precision=precision)
    o.precond = _PRECONDS[precond]
    out = ctypes.c_size_t()
    st = load().bmr_workspace_bytes(int(n), int(nnz), int(p), ctypes.byref(o), ctypes.byref(out))
    if st != 0:
        raise BmrError(st, "bmr_workspace_bytes")
    return int(out.value)


@dataclass
class SolveInfo:
    status: int
    band_iters: int
    block_iters: int
    n_replaced: int
    n_explicit_qr: int
    res_rec: np.ndarray
    time_ms: float
    hist: Optional[np.ndarray] = None
    kernel_ms: Optional[dict] = None   # mean ms per block iteration (profile=True)
    precision: str = "fp64"
    n_refine: int = 0                  # refinement cycles (precision="mixed")
    res_true: Optional[np.ndarray] = None  # final explicit relative residual (precision="mixed")
    res_explicit: Optional[np.ndarray] = None  # explicit ||b_i - A x_i|| / ||b_i|| of the returned X
    n_retained: int = 0                # removed candidates kept (retain=True)
    switch_iter: int = 0               # precision="relaxed": band iterations run in FP64 before the switch

    @property
    def status_name(self) -> str:
        return status_string(self.status)


class Ic0:
    """An IC(0) factor on the device (bmr_ic0_factor of M); holds its buffer."""

    def __init__(self, buf, n: int):
        self.buf = buf
        self.n = n

    @property
    def ptr(self) -> int:
        return self.buf.data_ptr()


def ic0_factor(M: DeviceCsr) -> Ic0:
    """Set up and factorise IC(0) of the symmetric matrix M on M's device."""
    import torch
    lib = load()
    need = ctypes.c_size_t()
    st = lib.bmr_ic0_bytes(M.n, M.nnz, ctypes.byref(need))
    if st != 0:
        raise BmrError(st, "bmr_ic0_bytes")
    buf = torch.empty(int(need.value), dtype=torch.uint8, device=M.val.device)
    Mc = M._c()
    st = lib.bmr_ic0_factor(ctypes.byref(Mc), buf.data_ptr(), buf.numel(), _stream_handle(M.val.device))
    if st != 0:
        raise BmrError(st, "bmr_ic0_factor")
    return Ic0(buf, M.n)


def ic0_apply(ic0: Ic0, V, trans: bool = False, W=None):
    """W = C^{-1} V (or C^{-T} V with trans) for the IC(0) factor C."""
    import torch
    _check_block(V, ic0.n, "V")
    if W is None:
        W = torch.empty_like(V)
    st = load().bmr_ic0_apply(ic0.ptr, V.data_ptr(), W.data_ptr(), int(V.shape[1]), int(bool(trans)),
                              _stream_handle(V.device))
    if st != 0:
        raise BmrError(st, "bmr_ic0_apply")
    return W


def solve(A: DeviceCsr, B, tol: float = 1e-8, max_iter: int = 10000, gamma: float = 1e-10, n_bench: int = 2,
          seed: int = 0, hist_cap: int = 0, poll_every: int = 0, X=None, workspace=None, check: bool = True,
          profile: bool = False, precision: str = "fp64", inner_tol: Optional[float] = None,
          max_refine: Optional[int] = None, ic0: Optional[Ic0] = None, retain: bool = False,
          accumulate: bool = False, relax_tol: Optional[float] = None):
    """Solve A X = B (A symmetric) by band-Lanczos block MINRES on the GPU.

    B: contiguous float64 (n, p) CUDA tensor.  Returns (X, SolveInfo).
    precision="mixed" runs the FP32 inner solver inside FP64 iterative
    refinement (inner_tol, max_refine: see bmr_opts_t); its hist rows are the
    explicit relative residuals after each refinement cycle.  precision=
    "relaxed" runs one solve in FP64 until every recurrence residual is below
    relax_tol (default min(1e-2, 1e3 tol)), then in FP32 (BMR_PREC_RELAXED).  ``retain``
    keeps removed candidates (BMR_FLAG_RETAIN), ``accumulate`` applies the
    previous blocks' rotations as accumulated matrices (BMR_FLAG_ACCUMULATE).
    With ``ic0``
    (from ic0_factor) the solve is split-preconditioned (bmr_solve_ic0; the
    history and res_rec then refer to the preconditioned residual).
    Errors (negative status) raise BmrError when ``check`` is true.
    """
    import torch
    lib = load()
    n = A.n
    _check_block(B, n, "B")
    p = int(B.shape[1])
    if X is None:
        X = torch.empty_like(B)
    _check_block(X, n, "X")
    o = _opts(tol, max_iter, gamma, n_bench, seed, hist_cap, poll_every,
              (FLAG_PROFILE if profile else 0) | (FLAG_RETAIN if retain else 0)
              | (FLAG_ACCUMULATE if accumulate else 0),
              precision, inner_tol, max_refine, relax_tol)
    if ic0 is not None:
        o.precond = PRECOND_IC0
    need = ctypes.c_size_t()
    st = lib.bmr_workspace_bytes(n, A.nnz, p, ctypes.byref(o), ctypes.byref(need))
    if st != 0:
        if check:
            raise BmrError(st, "bmr_workspace_bytes")
        return X, SolveInfo(st, 0, 0, 0, 0, np.zeros(p), 0.0)
    if workspace is None:
        workspace = torch.empty(int(need.value), dtype=torch.uint8, device=B.device)
    hist = np.zeros((max(hist_cap, 0), p)) if hist_cap > 0 else None
    stats = _Stats()
    Ac = A._c()
    hp = hist.ctypes.data if hist is not None else None
    if ic0 is not None:
        st = lib.bmr_solve_ic0(ctypes.byref(Ac), ic0.ptr, B.data_ptr(), X.data_ptr(), p, ctypes.byref(o),
                               workspace.data_ptr(), workspace.numel(), _stream_handle(B.device),
                               ctypes.byref(stats), hp)
    else:
        st = lib.bmr_solve(ctypes.byref(Ac), B.data_ptr(), X.data_ptr(), p, ctypes.byref(o), workspace.data_ptr(),
                           workspace.numel(), _stream_handle(B.device), ctypes.byref(stats), hp)
    if st < 0 and check:
        raise BmrError(st, "bmr_solve")
    info = SolveInfo(int(stats.status), int(stats.band_iters), int(stats.block_iters), int(stats.n_replaced),
                     int(stats.n_explicit_qr), np.array(stats.res_rec[:p]), float(stats.time_ms))
    info.precision = precision
    info.res_explicit = np.array(stats.res_explicit[:p])
    info.n_retained = int(stats.n_retained)
    info.switch_iter = int(stats.switch_iter)
    if precision == "mixed":
        info.n_refine = int(stats.n_refine)
        info.res_true = np.array(stats.res_true[:p])
    if hist is not None:
        info.hist = hist[:min(info.n_refine if precision == "mixed" else info.band_iters, hist_cap)]
    if profile:
        info.kernel_ms = dict(zip(KERNEL_NAMES, list(stats.t_kernel_ms)))
        info.kernel_ms["n_block_iters"] = int(stats.n_profiled)
    return X, info


def spmm(A: DeviceCsr, V, W=None):
    """W = A V for a contiguous float64 (n, p) CUDA tensor V (asynchronous)."""
    import torch
    _check_block(V, A.n, "V")
    if W is None:
        W = torch.empty_like(V)
    Ac = A._c()
    st = load().bmr_spmm(ctypes.byref(Ac), V.data_ptr(), W.data_ptr(), int(V.shape[1]), _stream_handle(V.device))
    if st != 0:
        raise BmrError(st, "bmr_spmm")
    return W


def spmm_f32(A: DeviceCsr, val32, V, W=None):
    """W = A V in FP32: A's structure with the float32 values val32 (CUDA
    tensor, nnz entries), V a contiguous float32 (n, p) CUDA tensor."""
    import torch
    _check_block(V, A.n, "V", torch.float32)
    if not (isinstance(val32, torch.Tensor) and val32.is_cuda and val32.dtype == torch.float32
            and val32.numel() == A.nnz and val32.is_contiguous()):
        raise ValueError("val32 must be a contiguous float32 CUDA tensor with nnz entries")
    if W is None:
        W = torch.empty_like(V)
    _check_block(W, A.n, "W", torch.float32)
    Ac = A._c()
    st = load().bmr_spmm_f32(ctypes.byref(Ac), val32.data_ptr(), V.data_ptr(), W.data_ptr(), int(V.shape[1]),
                             _stream_handle(V.device))
    if st != 0:
        raise BmrError(st, "bmr_spmm_f32")
    return W


def pattern_grad(A: DeviceCsr, Lam, X, out=None):
    """grad[e] = -(Lam_i . X_j + Lam_j . X_i) / 2 for every stored entry
    e = (i, j) of A: the symmetrised gradient on A's pattern of a loss whose
    adjoint solution is Lam (asynchronous)."""
    import torch
    _check_block(Lam, A.n, "Lam")
    _check_block(X, A.n, "X")
    if Lam.shape != X.shape:
        raise ValueError("Lam and X must have the same shape")
    if out is None:
        out = torch.empty(A.nnz, dtype=torch.float64, device=X.device)
    Ac = A._c()
    st = load().bmr_pattern_grad(ctypes.byref(Ac), Lam.data_ptr(), X.data_ptr(), int(X.shape[1]), out.data_ptr(),
                                 _stream_handle(X.device))
    if st != 0:
        raise BmrError(st, "bmr_pattern_grad")
    return out


def residual(A: DeviceCsr, B, X, want_R: bool = False, workspace=None):
    """Column norms ||b_i - A x_i|| (and R = B - A X if want_R)."""
    import torch
    _check_block(B, A.n, "B")
    _check_block(X, A.n, "X")
    p = int(B.shape[1])
    if workspace is None:
        workspace = torch.empty(workspace_bytes(A.n, p), dtype=torch.uint8, device=B.device)
    R = torch.empty_like(B) if want_R else None
    norms = (ctypes.c_double * p)()
    Ac = A._c()
    st = load().bmr_residual(ctypes.byref(Ac), B.data_ptr(), X.data_ptr(), p, R.data_ptr() if R is not None else None,
                             norms, workspace.data_ptr(), workspace.numel(), _stream_handle(B.device))
    if st != 0:
        raise BmrError(st, "bmr_residual")
    out = np.array(norms[:p])
    return (out, R) if want_R else out
