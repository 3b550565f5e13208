"""GeNIOS inexact-ADMM hot path on MI355X: Python binding of libgenios.so.

Every function here only marshals arguments (torch tensors -> device
pointers, the current HIP stream, a caller-owned workspace) and calls the C ABI
declared in include/genios.h.  All arithmetic runs in the library's HIP
kernels; importing this package fails if the library has not been built.

Functions
---------
lasso_solve, logreg_solve, huber_solve, boxls_solve
                               the solvers (Sec. 3.1 / Sec. 4.1 Lasso, Sec. 4.2 logistic,
                               Sec. 4.3 Huber fitting, Sec. 4.5 bounded least squares)
nystrom_build, nystrom_apply   the randomized Nystrom preconditioner (Sec. 2.2)
lasso_backward, GeniosLasso    adjoint of the Lasso solution map (torch.autograd.Function)
matvec, cast_bf16, gaussian_matrix, admm_update   single-kernel entry points
"""
from __future__ import annotations

import ctypes as C

import numpy as np
import torch

from . import _abi
from ._abi import GeniosError, Info

__all__ = ["lasso_solve", "logreg_solve", "huber_solve", "boxls_solve", "nystrom_build", "nystrom_apply", "lasso_backward",
           "GeniosLasso", "lasso", "matvec", "cast_bf16", "gaussian_matrix", "admm_update",
           "workspace_size", "make_opts", "GeniosError", "hvp_noalloc"]

_lib = _abi.load()


def _ptr(t: torch.Tensor | None) -> int | None:
    return None if t is None else t.data_ptr()


def _stream(dev: torch.device) -> int:
    return torch.cuda.current_stream(dev).cuda_stream


def _check_vec(t: torch.Tensor, name: str, dtype: torch.dtype, numel: int, dev):
    if not isinstance(t, torch.Tensor) or t.device != dev or t.dtype != dtype:
        raise TypeError(f"{name} must be a {dtype} tensor on {dev}")
    if not t.is_contiguous() or t.numel() != numel:
        raise ValueError(f"{name} must be contiguous with {numel} elements")


def _matrix(A: torch.Tensor, A16: torch.Tensor | None = None) -> _abi.Matrix:
    if not A.is_cuda:
        raise TypeError("A must be a GPU tensor")
    if A.dtype not in (torch.float32, torch.float64):
        raise TypeError("A must be float32 or float64 (the master copy)")
    if A.dim() not in (2, 3) or A.stride(-1) != 1:
        raise ValueError("A must be (m, n) or (batch, m, n) with unit column stride")
    M = _abi.Matrix()
    M.m, M.n = A.shape[-2], A.shape[-1]
    M.lda = A.stride(-2)
    M.batch = 1 if A.dim() == 2 else A.shape[0]
    M.stride_A = 0 if A.dim() == 2 else A.stride(0)
    M.hi_dtype = _abi.DT_F64 if A.dtype == torch.float64 else _abi.DT_F32
    M.A_hi = A.data_ptr()
    if A16 is not None:
        if A16.dtype not in (torch.bfloat16, torch.int16, torch.uint16) or A16.shape != A.shape \
                or A16.stride() != A.stride() or A16.device != A.device:
            raise ValueError("A16 must be a 16-bit tensor with A's shape, strides and device")
        M.A_bf16 = A16.data_ptr()
    return M


def make_opts(dtype: torch.dtype = torch.float32, **kw) -> _abi.Opts:
    """genios_opts with the paper's defaults, overridden by keyword arguments."""
    o = _abi.default_opts()
    prec = kw.pop("precision", "f64" if dtype == torch.float64 else "bf16_refine")
    o.precision = _abi.PRECISIONS[prec] if isinstance(prec, str) else int(prec)
    if "eps" in kw:
        e = kw.pop("eps")
        o.eps_abs = o.eps_rel = e
    for k, v in kw.items():
        if not hasattr(o, k) or k in ("struct_size", "workspace", "workspace_bytes", "stream",
                                      "history", "history_cap"):
            raise TypeError(f"unknown option {k!r}")
        setattr(o, k, int(v) if isinstance(v, bool) else v)
    return o


def workspace_size(op: int, M: _abi.Matrix, o: _abi.Opts) -> int:
    return int(_lib.genios_workspace_size(op, C.byref(M), C.byref(o)))


def _attach_workspace(o: _abi.Opts, nbytes: int, dev) -> torch.Tensor:
    ws = torch.empty(nbytes + 256, dtype=torch.uint8, device=dev)
    off = (-ws.data_ptr()) % 256
    o.workspace = ws.data_ptr() + off
    o.workspace_bytes = nbytes
    o.stream = _stream(dev)
    return ws


def _infos(arr, batch):
    return [arr[i].as_dict() for i in range(batch)]


def _bound(v, shape, dtype, dev, name):
    """None (unbounded), a scalar, or a tensor of the solution's shape -> device tensor or None."""
    if v is None:
        return None
    if isinstance(v, (int, float)):
        return torch.full(shape, float(v), dtype=dtype, device=dev)
    t = torch.as_tensor(v, dtype=dtype, device=dev)
    try:
        return torch.broadcast_to(t, shape).contiguous()
    except RuntimeError as e:
        raise ValueError(f"{name} must broadcast to {tuple(shape)}") from e


def _solve(kind, A, vec, lam, rho, A16, x0, z0, u0, history, box=None, **kw):
    dev = A.device
    M = _matrix(A, A16)
    o = make_opts(A.dtype, **kw)
    B, m, n = M.batch, M.m, M.n
    _check_vec(vec, "y" if kind == "logreg" else "b", A.dtype, B * m, dev)
    lam_h = np.ascontiguousarray(np.broadcast_to(np.asarray(lam, dtype=np.float64), (B,)))
    shape = (n,) if A.dim() == 2 else (B, n)
    if x0 is not None:
        x, z, u = (t.detach().clone().contiguous() for t in (x0, z0, u0))
        o.warm_start = 1
    else:
        x = torch.empty(shape, dtype=A.dtype, device=dev)
        z = torch.empty_like(x)
        u = torch.empty_like(x)
    hist = None
    if history:
        hist = np.zeros((B, int(history), _abi.HIST_FIELDS))
        o.history = hist.ctypes.data_as(C.POINTER(C.c_double))
        o.history_cap = int(history)
    op = {"lasso": _abi.OP_LASSO, "logreg": _abi.OP_LOGREG, "huber": _abi.OP_HUBER,
          "boxls": _abi.OP_BOXLS}[kind]
    ws = _attach_workspace(o, workspace_size(op, M, o), dev)
    infos = (Info * B)()
    fn = getattr(_lib, f"genios_{kind}_solve")
    if kind == "boxls":
        lo = _bound(box[0], shape, A.dtype, dev, "lo")
        hi = _bound(box[1], shape, A.dtype, dev, "hi")
        rc = fn(C.byref(M), _ptr(vec), _ptr(lo) if lo is not None else None,
                _ptr(hi) if hi is not None else None, float(rho), C.byref(o), _ptr(x), _ptr(z),
                _ptr(u), infos)
    else:
        rc = fn(C.byref(M), _ptr(vec), lam_h.ctypes.data_as(C.POINTER(C.c_double)), float(rho),
                C.byref(o), _ptr(x), _ptr(z), _ptr(u), infos)
    del ws
    if rc < 0:
        raise GeniosError(rc, f"genios_{kind}_solve")
    out = dict(x=x, z=z, u=u, info=_infos(infos, B), status=rc)
    if hist is not None:
        out["history"] = hist
    return out


def lasso_solve(A, b, lam, rho=1.0, A16=None, x0=None, z0=None, u0=None, history=0, **kw):
    """Lasso (1/2)||Ax - b||^2 + lam ||x||_1 by GeNIOS's inexact ADMM.

    A: (m, n) or (batch, m, n) float32/float64 GPU tensor; b: matching m-vectors.
    Returns dict(x, z, u, info=[per-problem dict], status[, history]).
    Keyword options are genios_opts fields (precision='f32'|'bf16_refine'|
    'bf16_only'|'f64', eps, max_iter, sketch_rank, ...).
    """
    return _solve("lasso", A, b, lam, rho, A16, x0, z0, u0, history, **kw)


def logreg_solve(A, y, lam, rho=1.0, A16=None, x0=None, z0=None, u0=None, history=0, **kw):
    """l1-logistic regression sum log(1 + exp(-y_i a_i^T x)) + lam ||x||_1 (labels +-1)."""
    return _solve("logreg", A, y, lam, rho, A16, x0, z0, u0, history, **kw)


def huber_solve(A, b, lam, rho=1.0, A16=None, x0=None, z0=None, u0=None, history=0, **kw):
    """l1-regularised Huber fitting sum l(a_i^T x - b_i) + lam ||x||_1, l(r) = r^2 for
    |r| <= huber_delta (default 1), 2 delta |r| - delta^2 beyond (Sec. 4.3)."""
    return _solve("huber", A, b, lam, rho, A16, x0, z0, u0, history, **kw)


def boxls_solve(A, b, lo=0.0, hi=1.0, rho=1.0, A16=None, x0=None, z0=None, u0=None, history=0,
                **kw):
    """Box-constrained least squares (1/2)||Ax - b||^2, lo <= x <= hi (Sec. 4.5 through the
    QP form of Sec. 3.2).  lo/hi: None (unbounded), a scalar or a tensor of x's shape."""
    return _solve("boxls", A, b, 0.0, rho, A16, x0, z0, u0, history, box=(lo, hi), **kw)


def nystrom_build(A, s, d=None, omega=None, A16=None, **kw):
    """Rank-s Nystrom approximation of A^T diag(d) A: returns (U (n x s col-major), lamhat, info).

    U is returned as a (batch, s, n) tensor whose row j is column j of U.
    """
    dev = A.device
    M = _matrix(A, A16)
    o = make_opts(A.dtype, **kw)
    o.sketch_rank = int(s)
    B, m, n = M.batch, M.m, M.n
    if d is not None:
        _check_vec(d, "d", A.dtype, B * m, dev)
    if omega is not None:
        if omega.dtype != A.dtype or not omega.is_contiguous() or omega.numel() != B * n * s:
            raise ValueError("omega must be contiguous (batch, s, n) rows = columns of Omega")
    U = torch.empty((B, s, n), dtype=A.dtype, device=dev)
    lamhat = torch.empty((B, s), dtype=torch.float64, device=dev)
    ws = _attach_workspace(o, workspace_size(_abi.OP_NYSTROM, M, o), dev)
    infos = (Info * B)()
    rc = _lib.genios_nystrom_build(C.byref(M), _ptr(d), int(s), _ptr(omega), C.byref(o), _ptr(U),
                                   _ptr(lamhat), infos)
    del ws
    if rc < 0:
        raise GeniosError(rc, "genios_nystrom_build")
    return U, lamhat, _infos(infos, B)


def nystrom_apply(U, lamhat, nu, r):
    """z = P^-1 r for the factored preconditioner; U (batch, s, n), lamhat (batch, s), r (batch, n)."""
    dev = U.device
    B, s, n = U.shape
    o = _abi.default_opts()
    _check_vec(r, "r", U.dtype, B * n, dev)
    z = torch.empty_like(r)
    nb = (n + 1023) // 1024
    need = B * nb * (128 + 16) * 8 + B * 16 * 4 + B * 128 * 8 + B * 64 + 4096
    ws = _attach_workspace(o, need, dev)
    rc = _lib.genios_nystrom_apply(n, s, B, _abi.DT_F64 if U.dtype == torch.float64 else _abi.DT_F32,
                                   _ptr(U), _ptr(lamhat), float(nu), _ptr(r), _ptr(z), C.byref(o))
    del ws
    if rc < 0:
        raise GeniosError(rc, "genios_nystrom_apply")
    return z


def lasso_backward(A, z_star, grad_z, lam, A16=None, **kw):
    """(grad_b, grad_lam) of a loss through the Lasso solution map (implicit differentiation)."""
    dev = A.device
    M = _matrix(A, None)
    kw.setdefault("precision", "f64" if A.dtype == torch.float64 else "f32")
    kw.setdefault("max_cg_iter", 1000)
    o = make_opts(A.dtype, **kw)
    B, m, n = M.batch, M.m, M.n
    _check_vec(z_star, "z_star", A.dtype, B * n, dev)
    _check_vec(grad_z, "grad_z", A.dtype, B * n, dev)
    lam_h = np.ascontiguousarray(np.broadcast_to(np.asarray(lam, dtype=np.float64), (B,)))
    grad_b = torch.empty((m,) if A.dim() == 2 else (B, m), dtype=A.dtype, device=dev)
    grad_lam = np.zeros(B)
    ws = _attach_workspace(o, workspace_size(_abi.OP_BACKWARD, M, o), dev)
    infos = (Info * B)()
    rc = _lib.genios_lasso_backward(C.byref(M), _ptr(z_star), _ptr(grad_z),
                                    lam_h.ctypes.data_as(C.POINTER(C.c_double)), C.byref(o),
                                    _ptr(grad_b), grad_lam.ctypes.data_as(C.POINTER(C.c_double)),
                                    infos)
    del ws
    if rc < 0:
        raise GeniosError(rc, "genios_lasso_backward")
    return grad_b, torch.from_numpy(grad_lam), _infos(infos, B)


class GeniosLasso(torch.autograd.Function):
    """z* = argmin (1/2)||A x - b||^2 + lam ||x||_1, differentiable in b and lam."""

    @staticmethod
    def forward(ctx, A, b, lam, A16=None, opts=None):
        opts = dict(opts or {})
        lam_t = torch.as_tensor(lam, dtype=torch.float64).detach().cpu()
        out = lasso_solve(A, b.detach(), lam_t.numpy(), A16=A16, **opts)
        z = out["z"]
        ctx.save_for_backward(A, z)
        ctx.lam = lam_t
        ctx.lam_shape = torch.as_tensor(lam).shape
        ctx.info = out["info"]
        return z

    @staticmethod
    def backward(ctx, grad_z):
        A, z = ctx.saved_tensors
        grad_b, grad_lam, _ = lasso_backward(A, z, grad_z.contiguous(), ctx.lam.numpy())
        gl = grad_lam.to(dtype=torch.float64).reshape(ctx.lam_shape) if len(ctx.lam_shape) else \
            grad_lam.to(dtype=torch.float64).sum()
        return None, grad_b, gl, None, None


def lasso(A, b, lam, A16=None, **opts):
    return GeniosLasso.apply(A, b, lam, A16, opts)


def matvec(A, v, trans=False, A16=None):
    """A v (trans=False) or A^T v with the library's product kernels."""
    dev = A.device
    M = _matrix(A, A16)
    o = _abi.default_opts()
    o.precision = _abi.PREC_BF16_ONLY if A16 is not None else (
        _abi.PREC_F64 if A.dtype == torch.float64 else _abi.PREC_F32)
    B, m, n = M.batch, M.m, M.n
    _check_vec(v, "v", A.dtype, B * (m if trans else n), dev)
    out = torch.empty((B, n if trans else m) if A.dim() == 3 else (n if trans else m,),
                      dtype=A.dtype, device=dev)
    ws = _attach_workspace(o, workspace_size(_abi.OP_MATVEC, M, o), dev)
    rc = _lib.genios_matvec(C.byref(M), int(bool(trans)), int(A16 is not None), _ptr(v), _ptr(out),
                            C.byref(o))
    del ws
    if rc < 0:
        raise GeniosError(rc, "genios_matvec")
    return out


def hvp(A, p, d=None, A16=None, batch_mfma=1):
    """A^T diag(d) A p (d None: A^T A p) with the CG loop's product kernels.  A batch
    sharing one matrix (A.expand(B, m, n)) with BF16 A16 uses the matrix-core products
    for all problems at once unless batch_mfma = 0 (see genios_opts.batch_mfma)."""
    dev = A.device
    M = _matrix(A, A16)
    o = _abi.default_opts()
    o.batch_mfma = int(batch_mfma)
    o.precision = _abi.PREC_BF16_ONLY if A16 is not None else (
        _abi.PREC_F64 if A.dtype == torch.float64 else _abi.PREC_F32)
    B, m, n = M.batch, M.m, M.n
    _check_vec(p, "p", A.dtype, B * n, dev)
    if d is not None:
        _check_vec(d, "d", A.dtype, B * m, dev)
    out = torch.empty((B, n) if A.dim() == 3 else (n,), dtype=A.dtype, device=dev)
    ws = _attach_workspace(o, workspace_size(_abi.OP_HVP, M, o), dev)
    rc = _lib.genios_hvp(C.byref(M), int(A16 is not None), _ptr(d), _ptr(p), _ptr(out),
                         C.byref(o))
    del ws
    if rc < 0:
        raise GeniosError(rc, "genios_hvp")
    return out


def hvp_noalloc(A, p, d=None, A16=None, out=None, batch_mfma=1):
    """``hvp`` through genios_hvp_noalloc: no workspace is allocated (the library's
    static per-GPU scratch holds the partial sums); ``out`` may be given so that
    the call allocates nothing at all."""
    dev = A.device
    M = _matrix(A, A16)
    o = _abi.default_opts()
    o.batch_mfma = int(batch_mfma)
    o.precision = _abi.PREC_BF16_ONLY if A16 is not None else (
        _abi.PREC_F64 if A.dtype == torch.float64 else _abi.PREC_F32)
    B, m, n = M.batch, M.m, M.n
    _check_vec(p, "p", A.dtype, B * n, dev)
    if d is not None:
        _check_vec(d, "d", A.dtype, B * m, dev)
    if out is None:
        out = torch.empty((B, n) if A.dim() == 3 else (n,), dtype=A.dtype, device=dev)
    else:
        _check_vec(out, "out", A.dtype, B * n, dev)
    o.stream = _stream(dev)
    rc = _lib.genios_hvp_noalloc(C.byref(M), int(A16 is not None), _ptr(d), _ptr(p), _ptr(out),
                                 C.byref(o))
    if rc < 0:
        raise GeniosError(rc, "genios_hvp_noalloc")
    return out


STREAM_READ_SCRATCH = 4096  # GENIOS_STREAM_READ_SCRATCH


def stream_read_seconds(t: torch.Tensor, reps: int = 10) -> float:
    """HIP-event time of `reps` plain streaming reads of tensor t's bytes (the
    HBM read-rate reference for the bandwidth-bound kernels)."""
    if not t.is_cuda or not t.is_contiguous():
        raise TypeError("stream_read needs a contiguous GPU tensor")
    scratch = torch.empty(STREAM_READ_SCRATCH, dtype=torch.int32, device=t.device)
    o = _abi.default_opts()
    o.stream = _stream(t.device)
    sec = C.c_double(0.0)
    nbytes = t.numel() * t.element_size() // 16 * 16
    rc = _lib.genios_stream_read(_ptr(t), nbytes, int(reps), _ptr(scratch), C.byref(sec), C.byref(o))
    if rc < 0:
        raise GeniosError(rc, "genios_stream_read")
    return sec.value


def cast_bf16(A: torch.Tensor) -> torch.Tensor:
    """Round-to-nearest-even BF16 copy of an FP32 tensor (returned as torch.bfloat16)."""
    if A.dtype != torch.float32 or not A.is_contiguous() or not A.is_cuda:
        raise TypeError("cast_bf16 needs a contiguous float32 GPU tensor")
    out = torch.empty(A.shape, dtype=torch.bfloat16, device=A.device)
    o = _abi.default_opts()
    o.stream = _stream(A.device)
    rc = _lib.genios_cast_bf16(_ptr(A), _ptr(out), A.numel(), C.byref(o))
    if rc < 0:
        raise GeniosError(rc, "genios_cast_bf16")
    return out


def gaussian_matrix(n, s, seed, stream_id=0, device="cuda"):
    """The sketch's n x s standard-normal test matrix, returned as (s, n) rows = columns."""
    out = torch.empty((s, n), dtype=torch.float32, device=device)
    o = _abi.default_opts()
    o.stream = _stream(out.device)
    rc = _lib.genios_gaussian_matrix(int(n), int(s), int(seed), int(stream_id), _ptr(out),
                                     C.byref(o))
    if rc < 0:
        raise GeniosError(rc, "genios_gaussian_matrix")
    return out


def admm_update(x, z, u, alpha, kappa):
    """Fused over-relaxed prox / dual update (in place on z, u); returns the four FP64 norms."""
    dev = x.device
    n = x.numel()
    for t, nm in ((z, "z"), (u, "u")):
        _check_vec(t, nm, x.dtype, n, dev)
    o = _abi.default_opts()
    need = ((n + 1023) // 1024) * (128 + 16) * 8 + 4096
    ws = _attach_workspace(o, need, dev)
    norms = np.zeros(4)
    rc = _lib.genios_admm_update(n, _abi.DT_F64 if x.dtype == torch.float64 else _abi.DT_F32,
                                 float(alpha), float(kappa), _ptr(x), _ptr(z), _ptr(u),
                                 norms.ctypes.data_as(C.POINTER(C.c_double)), C.byref(o))
    del ws
    if rc < 0:
        raise GeniosError(rc, "genios_admm_update")
    return norms
