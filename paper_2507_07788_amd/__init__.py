"""Python binding of libsqr: shifted Cholesky QR (CholQR3) and the Cholesky QR
block append on AMD MI355X (arXiv 2507.07788, Algorithms 1-3).

Argument marshalling only: every step of the method runs in the HIP kernels of
libsqr.so.  Tensors are torch FP64 CUDA (HIP) tensors holding column-major
matrices, i.e. a matrix of shape (m, n) with strides (1, ld), ld >= m; use
``colmajor`` to allocate one.  Loading fails loudly when libsqr.so is missing.
"""
from __future__ import annotations

import ctypes
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libsqr.so")

SQR_OK, SQR_NOT_CONVERGED, SQR_BREAKDOWN, SQR_ENONFINITE = 0, 1, 2, 3
SQR_ENULL, SQR_EDIM, SQR_EHIP, SQR_EOPT, SQR_ELIMIT = -1, -2, -3, -4, -5


class SqrOpts(ctypes.Structure):
    _fields_ = [("precision", ctypes.c_int32), ("first_pass_shift", ctypes.c_int32),
                ("min_passes", ctypes.c_int32), ("max_iter", ctypes.c_int32),
                ("tol", ctypes.c_double), ("unit_roundoff", ctypes.c_double),
                ("max_escalations", ctypes.c_int32), ("power_steps", ctypes.c_int32),
                ("shift_policy", ctypes.c_int32), ("append_shift_dim", ctypes.c_int32)]

#: option sets of the Cholesky QR variants of Sec. 3.1 (shift_policy 0:
#: Algorithm 1's recomputed shift, 1: none, 2: isCholQR's fixed shift)
VARIANTS = {
    "CholQR": dict(first_pass_shift=0, min_passes=1, max_iter=1, shift_policy=1),
    "CholQR2": dict(first_pass_shift=0, min_passes=2, max_iter=2, shift_policy=1),
    "sCholQR3": dict(first_pass_shift=1, min_passes=3, max_iter=3, shift_policy=1),
    "isCholQR": dict(first_pass_shift=0, min_passes=0, max_iter=10, shift_policy=2),
    "rsCholQR": dict(first_pass_shift=0, min_passes=0, max_iter=10, shift_policy=0),
    "CholQR3": dict(first_pass_shift=1, min_passes=3, max_iter=10, shift_policy=0),
}


class SqrInfo(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("passes", ctypes.c_int32),
                ("chol_attempts", ctypes.c_int32), ("converged", ctypes.c_int32),
                ("orth_fro", ctypes.c_double), ("sigma", ctypes.c_double * 16)]

    def as_dict(self) -> dict:
        n = min(self.passes, 16)
        return dict(status=self.status, passes=self.passes,
                    chol_attempts=self.chol_attempts, converged=self.converged,
                    orth_fro=self.orth_fro, sigma=list(self.sigma[:n]))


class SqrBatchItem(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("rc", ctypes.c_int32), ("basis", ctypes.c_void_p),
                ("inp", ctypes.c_void_p), ("ld_in", ctypes.c_int64), ("m", ctypes.c_int64),
                ("cols", ctypes.c_int64), ("cap", ctypes.c_int64), ("Q", ctypes.c_void_p),
                ("ldq", ctypes.c_int64), ("R", ctypes.c_void_p), ("ldr", ctypes.c_int64),
                ("info", SqrInfo)]


SQR_BATCH_ORTH, SQR_BATCH_APPEND = 0, 1


class SqrProf(ctypes.Structure):
    _fields_ = [("launches", ctypes.c_int64 * 2), ("ms", ctypes.c_double * 2),
                ("bytes", ctypes.c_double * 2)]


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"libsqr.so is not built ({LIB_PATH}); run "
                          "`python -m paper_2507_07788_amd.build` first")
    lib = ctypes.CDLL(LIB_PATH)
    P, I64, I32 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int
    lib.sqr_default_opts.argtypes = [ctypes.POINTER(SqrOpts)]
    lib.sqr_default_opts.restype = None
    lib.sqr_orth.argtypes = [ctypes.POINTER(P), ctypes.POINTER(SqrOpts), I64, I64, P, I64,
                             P, I64, I64, P, I64, P, ctypes.POINTER(SqrInfo)]
    lib.sqr_orth.restype = I32
    lib.sqr_orth_noalloc.argtypes = [ctypes.POINTER(SqrOpts), I64, I64, P, I64, P, I64,
                                     P, I64, P, ctypes.POINTER(SqrInfo)]
    lib.sqr_orth_noalloc.restype = I32
    lib.sqr_panel.argtypes = [ctypes.POINTER(P), ctypes.POINTER(SqrOpts), I64, I64, P, I64, I64,
                              P, I64, I64, P, I64, P, ctypes.POINTER(SqrInfo)]
    lib.sqr_panel.restype = I32
    lib.sqr_batch.argtypes = [ctypes.POINTER(SqrOpts), ctypes.POINTER(SqrBatchItem), ctypes.c_int32, P]
    lib.sqr_batch.restype = I32
    lib.sqr_append.argtypes = [P, P, I64, I64, P, ctypes.POINTER(SqrInfo)]
    lib.sqr_append.restype = I32
    lib.sqr_last_info.argtypes = [P, ctypes.POINTER(SqrInfo)]
    lib.sqr_last_info.restype = I32
    lib.sqr_cols.argtypes = [P]
    lib.sqr_cols.restype = I64
    lib.sqr_free.argtypes = [P]
    lib.sqr_free.restype = None
    lib.sqr_park.argtypes = [P]
    lib.sqr_park.restype = I32
    lib.sqr_prof_enable.argtypes = [I32]
    lib.sqr_prof_enable.restype = None
    lib.sqr_prof_read.argtypes = [ctypes.POINTER(SqrProf)]
    lib.sqr_prof_read.restype = I32
    return lib


lib = _load()


def sqr_default_opts(**overrides) -> SqrOpts:
    o = SqrOpts()
    lib.sqr_default_opts(ctypes.byref(o))
    for k, v in overrides.items():
        setattr(o, k, v)
    return o


def colmajor(m: int, n: int, ld: int | None = None, device="cuda",
             dtype=torch.float64) -> torch.Tensor:
    """Uninitialised column-major (m, n) tensor with leading dimension ld."""
    ld = m if ld is None else ld
    return torch.empty((n, ld), dtype=dtype, device=device).t()[:m]


def _ld(t: torch.Tensor) -> int:
    if t.dtype != torch.float64 or not t.is_cuda:
        raise TypeError("expected a float64 GPU tensor")
    if t.dim() != 2 or (t.shape[0] > 1 and t.stride(0) != 1):
        raise ValueError("expected a column-major matrix (stride(0) == 1)")
    return max(t.stride(1), t.shape[0]) if t.shape[1] > 1 else max(t.shape[0], 1)


def _stream(stream) -> int:
    if stream is not None:
        return stream.cuda_stream
    # the raw handle of the current device's current stream (what
    # torch.cuda.current_stream().cuda_stream returns, without building a
    # Stream object on every call)
    return torch._C._cuda_getCurrentRawStream(torch.cuda.current_device())


class Basis:
    """A handle plus the tensors it borrows: Q (m x cap), R (cap x cap)."""

    def __init__(self, handle, Q, R, m, cap):
        self.handle, self.Q, self.R, self.m, self.cap = handle, Q, R, m, cap

    @property
    def n(self) -> int:
        return int(lib.sqr_cols(self.handle)) if self.handle else 0

    def q(self) -> torch.Tensor:
        return self.Q[:, :self.n]

    def r(self) -> torch.Tensor:
        return self.R[:self.n, :self.n]

    def __del__(self):
        if getattr(self, "handle", None):
            sqr_free(self)


def _check_matrix(name: str, t: torch.Tensor, rows: int, min_cols: int, device) -> None:
    """Shape and device of a caller buffer, before the library sees only its
    pointer and leading dimension."""
    if t.dim() != 2:
        raise ValueError(f"{name} must be a matrix")
    if t.device != device:
        raise ValueError(f"{name} is on {t.device}, expected {device}")
    if t.shape[0] != rows or t.shape[1] < min_cols:
        raise ValueError(f"{name} has shape {tuple(t.shape)}, expected ({rows}, >= {min_cols})")


def sqr_orth(A: torch.Tensor, cap: int | None = None, opts: SqrOpts | None = None,
             Q: torch.Tensor | None = None, R: torch.Tensor | None = None,
             stream=None, sync: bool = True):
    """Q R = A (Algorithm 1 with the CholQR3 start).  Returns (Basis, info
    dict or None); raises ValueError on inconsistent shapes or devices and
    RuntimeError on other usage errors (negative codes)."""
    if A.dim() != 2:
        raise ValueError("A must be a matrix")
    m, n = A.shape
    cap = n if cap is None else cap
    if cap < n:
        raise ValueError(f"cap = {cap} is below n = {n}")
    if Q is None:
        Q = colmajor(m, cap, device=A.device)
    if R is None:
        R = colmajor(cap, cap, device=A.device)
    _check_matrix("Q", Q, m, cap, A.device)
    _check_matrix("R", R, cap, cap, A.device)
    h = ctypes.c_void_p()
    info = SqrInfo()
    rc = lib.sqr_orth(ctypes.byref(h), ctypes.byref(opts) if opts is not None else None,
                      m, n, A.data_ptr(), _ld(A), Q.data_ptr(), _ld(Q), cap,
                      R.data_ptr(), _ld(R), _stream(stream),
                      ctypes.byref(info) if sync else None)
    if rc < 0:
        raise RuntimeError(f"sqr_orth failed with code {rc}")
    return Basis(h, Q, R, m, cap), (info.as_dict() if sync else None)


def sqr_panel(A: torch.Tensor, r: int, cap: int | None = None, opts: SqrOpts | None = None,
              Q: torch.Tensor | None = None, R: torch.Tensor | None = None, stream=None):
    """Algorithm 3 (the panel scheme): r panels of A appended in turn to an
    empty basis.  Returns (Basis, info of the last panel); raises ValueError
    on inconsistent shapes or devices and RuntimeError on other usage
    errors."""
    if A.dim() != 2:
        raise ValueError("A must be a matrix")
    m, n = A.shape
    cap = n if cap is None else cap
    if Q is None:
        Q = colmajor(m, cap, device=A.device)
    if R is None:
        R = colmajor(cap, cap, device=A.device)
    _check_matrix("Q", Q, m, cap, A.device)
    _check_matrix("R", R, cap, cap, A.device)
    h = ctypes.c_void_p()
    info = SqrInfo()
    rc = lib.sqr_panel(ctypes.byref(h), ctypes.byref(opts) if opts is not None else None,
                       m, n, A.data_ptr(), _ld(A), r, Q.data_ptr(), _ld(Q), cap,
                       R.data_ptr(), _ld(R), _stream(stream), ctypes.byref(info))
    if rc < 0:
        raise RuntimeError(f"sqr_panel failed with code {rc}")
    return Basis(h, Q, R, m, cap), info.as_dict()


def sqr_orth_noalloc(A: torch.Tensor, Q: torch.Tensor, R: torch.Tensor,
                     opts: SqrOpts | None = None, stream=None, sync: bool = True):
    """Q R = A into the caller's Q (m x n) and R (n x n) with the library's
    static per-GPU scratch (sqr_orth_noalloc: no device allocation, no
    handle).  Returns the info dict (sync) or None; raises ValueError on
    inconsistent shapes or devices and RuntimeError on other usage errors."""
    if A.dim() != 2:
        raise ValueError("A must be a matrix")
    m, n = A.shape
    _check_matrix("Q", Q, m, n, A.device)
    _check_matrix("R", R, n, n, A.device)
    info = SqrInfo()
    rc = lib.sqr_orth_noalloc(ctypes.byref(opts) if opts is not None else None,
                              m, n, A.data_ptr(), _ld(A), Q.data_ptr(), _ld(Q),
                              R.data_ptr(), _ld(R), _stream(stream),
                              ctypes.byref(info) if sync else None)
    if rc < 0:
        raise RuntimeError(f"sqr_orth_noalloc failed with code {rc}")
    return info.as_dict() if sync else None


def sqr_append(b: Basis, W: torch.Tensor, stream=None) -> dict:
    """Algorithm 2: append the columns of W to the basis.  Returns the info
    dict; raises ValueError on a W of the wrong height or device and
    RuntimeError on other usage errors."""
    _check_matrix("W", W, b.m, 1, b.Q.device)
    info = SqrInfo()
    rc = lib.sqr_append(b.handle, W.data_ptr(), W.shape[1], _ld(W), _stream(stream),
                        ctypes.byref(info))
    if rc < 0:
        raise RuntimeError(f"sqr_append failed with code {rc}")
    return info.as_dict()


def sqr_batch(calls, opts: SqrOpts | None = None, stream=None) -> list:
    """Run several calls together (sqr_batch): each entry is
    ``("orth", A, cap, Q, R)`` or ``("append", basis, W)``.  Returns, per
    call, a dict with ``rc`` (as sqr_orth / sqr_append return it), ``info``
    and, for an orthogonalisation that ran, its ``basis``.  Raises ValueError
    on inconsistent shapes or devices before the library is called."""
    items = (SqrBatchItem * len(calls))()
    keep = []
    for it, call in zip(items, calls):
        if call[0] == "orth":
            _, A, cap, Q, R = call
            if A.dim() != 2:
                raise ValueError("A must be a matrix")
            m, n = A.shape
            _check_matrix("Q", Q, m, cap, A.device)
            _check_matrix("R", R, cap, cap, A.device)
            it.kind, it.inp, it.ld_in, it.m, it.cols, it.cap = SQR_BATCH_ORTH, A.data_ptr(), _ld(A), m, n, cap
            it.Q, it.ldq, it.R, it.ldr = Q.data_ptr(), _ld(Q), R.data_ptr(), _ld(R)
            keep.append((A, Q, R))
        elif call[0] == "append":
            _, b, W = call
            _check_matrix("W", W, b.m, 1, b.Q.device)
            it.kind, it.basis, it.inp, it.ld_in, it.cols = SQR_BATCH_APPEND, b.handle.value, W.data_ptr(), _ld(W), W.shape[1]
            keep.append((W,))
        else:
            raise ValueError(f"unknown call kind {call[0]!r}")
    rc = lib.sqr_batch(ctypes.byref(opts) if opts is not None else None, items, len(calls), _stream(stream))
    if rc in (SQR_ENULL, SQR_EOPT):
        raise RuntimeError(f"sqr_batch failed with code {rc}")
    out = []
    for it, call in zip(items, calls):
        d = {"rc": it.rc, "info": it.info.as_dict()}
        if call[0] == "orth" and it.rc >= 0 and it.basis:
            _, A, cap, Q, R = call
            d["basis"] = Basis(ctypes.c_void_p(it.basis), Q, R, A.shape[0], cap)
        out.append(d)
    return out


def sqr_last_info(b: Basis) -> dict:
    info = SqrInfo()
    rc = lib.sqr_last_info(b.handle, ctypes.byref(info))
    if rc < 0:
        raise RuntimeError(f"sqr_last_info failed with code {rc}")
    return info.as_dict()


def sqr_free(b: Basis) -> None:
    if b.handle:
        lib.sqr_free(b.handle)
        b.handle = None


def sqr_park(b: Basis) -> None:
    """Return the handle's workspace to the library pool (sqr_park)."""
    if b.handle:
        rc = lib.sqr_park(b.handle)
        if rc < 0:
            raise RuntimeError(f"sqr_park failed with code {rc}")


def sqr_prof_enable(on: bool = True) -> None:
    """Record HIP events around every streaming-kernel launch (sqr_prof.h)."""
    lib.sqr_prof_enable(1 if on else 0)


def sqr_prof_read() -> dict:
    """Fold the recorded launches: {'gram'|'apply': (launches, ms, bytes)}."""
    pr = SqrProf()
    rc = lib.sqr_prof_read(ctypes.byref(pr))
    if rc < 0:
        raise RuntimeError(f"sqr_prof_read failed with code {rc}")
    return {"gram": (pr.launches[0], pr.ms[0], pr.bytes[0]),
            "apply": (pr.launches[1], pr.ms[1], pr.bytes[1])}
