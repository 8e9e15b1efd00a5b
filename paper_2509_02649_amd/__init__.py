"""Fourier-basis kernel ridge regression on MI355X (HIP, gfx950).

Thin Python layer over libfastkernel.so: argument checks and marshalling of
torch device tensors and the current HIP stream.  Every numerical step runs in
the library's kernels.  There is no CPU fallback: without the built library
(or without a HIP device) the functions raise.

The estimator (Sec. 2.1, eq. kenrel_reg of the paper):
    theta = (n^-1 Phi^* Phi + lambda P)^-1 n^-1 Phi^* Y
on the Fourier basis exp(i k.x), ||k||_inf <= m, with the Gram generator
M[q] = n^-1 sum_j exp(+i q.X_j) and b_k = n^-1 sum_j Y_j exp(-i k.X_j)
formed by type-1 NUFFTs (Sec. 2.3).
"""
from __future__ import annotations

import ctypes as C
import math
import threading
from typing import Optional, Sequence

import torch

from . import _lib
from ._lib import FkError, fk_fit_info, fk_penalty, fk_options, FK_F32, FK_F64, PEN

__all__ = ["Context", "gram", "restrict", "solve", "solve_workspace_size", "fit_kept_workspace_size", "solve_cg",
           "toeplitz_apply", "fit", "predict", "predict_noalloc", "heldout_mse", "fit_backward", "additive_gram",
           "additive_fit", "generate_uniform", "generate_targets", "KernelRidgeGridLoss", "FkError",
           "autotune_table", "autotune_load", "autotune_clear"]


def _stream_ptr(device):
    return C.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def _ptr(t: Optional[torch.Tensor]):
    return C.c_void_p(0 if t is None else t.data_ptr())


def _dtype_code(t: torch.Tensor) -> int:
    if t.dtype == torch.float32:
        return FK_F32
    if t.dtype == torch.float64:
        return FK_F64
    raise TypeError(f"points must be float32 or float64, got {t.dtype}")


def _dev_tensor(t: torch.Tensor, name: str) -> torch.Tensor:
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise ValueError(f"{name} must be a HIP device tensor")
    return t.contiguous()


class Context:
    """A library context bound to one device; enqueues on torch's current stream."""

    def __init__(self, device: int = 0, eps: float = 2e-7, max_refine: int = 8, refine_tol: float = 1e-10,
                 autotune: int = 0):
        if not torch.cuda.is_available():
            raise RuntimeError("no HIP device visible: libfastkernel needs an MI355X")
        self.lib = _lib.load()
        self.device = device
        h = C.c_void_p()
        _lib.check(self.lib.fk_create(C.byref(h), device, _stream_ptr(device)), "fk_create")
        self.h = h
        opt = fk_options(eps, max_refine, refine_tol, 1, autotune)
        _lib.check(self.lib.fk_set_options(self.h, C.byref(opt)), "fk_set_options")
        self._ws = None

    def __del__(self):
        try:
            if getattr(self, "h", None):
                self.lib.fk_destroy(self.h)
                self.h = None
        except Exception:
            pass

    def bind_stream(self):
        _lib.check(self.lib.fk_set_stream(self.h, _stream_ptr(self.device)), "fk_set_stream")

    def workspace(self, nbytes: int) -> torch.Tensor:
        """A cached device byte buffer of at least nbytes (256-byte aligned by the allocator)."""
        if self._ws is None or self._ws.numel() < nbytes:
            self._ws = None
            self._ws = torch.empty(int(nbytes), dtype=torch.uint8, device=f"cuda:{self.device}")
        return self._ws


_default: dict = {}


def default_context(device: int = 0) -> Context:
    ctx = _default.get(device)
    if ctx is None:
        ctx = Context(device)
        _default[device] = ctx
    return ctx


def _penalty(kind: str, s: float = 1.0, p: Optional[torch.Tensor] = None, mu: float = 0.0,
             box_lo=(-math.pi / 2, -math.pi / 2), box_hi=(math.pi / 2, math.pi / 2), alpha=None, coef=None):
    """The fk_penalty struct (and the host arrays it points to, to keep alive during the call).

    kind "pde_box": lambda diag(1 + ||k||^(2s)) + mu D^* C D for the operator sum_t coef[t] d^alpha[t]
    on the box [box_lo, box_hi] (radians; Sec. 4, tractable domains), alpha [nterms][d] integers."""
    pen = fk_penalty()
    pen.kind = PEN[kind]
    pen.s = float(s)
    keep = []
    if kind == "diag":
        arr = (C.c_double * p.numel())(*[float(v) for v in p.detach().cpu().double().tolist()])
        keep.append(arr)
        pen.p = C.cast(arr, C.POINTER(C.c_double))
    pen.mu = float(mu)
    lo = list(box_lo) + [0.0] * (2 - len(box_lo))
    hi = list(box_hi) + [0.0] * (2 - len(box_hi))
    pen.box_lo[0], pen.box_lo[1] = lo[:2]
    pen.box_hi[0], pen.box_hi[1] = hi[:2]
    if kind == "pde_box":
        flat = [int(v) for row in alpha for v in (row if hasattr(row, "__len__") else [row])]
        a = (C.c_int * len(flat))(*flat)
        c = (C.c_double * len(coef))(*[float(v) for v in coef])
        keep += [a, c]
        pen.nterms = len(coef)
        pen.alpha = C.cast(a, C.POINTER(C.c_int))
        pen.coef = C.cast(c, C.POINTER(C.c_double))
    return pen, keep


def _modes(m: int, d: int) -> int:
    return (2 * m + 1) ** d


def gram(X: torch.Tensor, Y: Optional[torch.Tensor], m: int, ctx: Optional[Context] = None, info: bool = False):
    """M [(4m+1)^d] complex128 and b [T, (2m+1)^d] complex128 from X [d, n], Y [T, n]."""
    ctx = ctx or default_context(X.device.index or 0)
    ctx.bind_stream()
    X = _dev_tensor(X, "X")
    d, n = X.shape
    T = 0 if Y is None else Y.shape[0]
    if Y is not None:
        Y = _dev_tensor(Y, "Y")
        if Y.dtype != X.dtype or Y.shape[1] != n:
            raise ValueError("Y must be [T, n] with the dtype of X")
    nb = C.c_size_t()
    _lib.check(ctx.lib.fk_gram_workspace_size(ctx.h, d, n, T, m, C.byref(nb)), "fk_gram_workspace_size")
    ws = ctx.workspace(nb.value)
    M = torch.empty(((4 * m + 1) ** d) * 2, dtype=torch.float64, device=X.device)
    b = torch.empty((max(T, 1), _modes(m, d) * 2), dtype=torch.float64, device=X.device)
    inf = fk_fit_info()
    _lib.check(ctx.lib.fk_gram(ctx.h, d, n, _dtype_code(X), _ptr(X), T, _ptr(Y), m, _ptr(M), _ptr(b), _ptr(ws),
                               nb.value, C.byref(inf)), "fk_gram")
    M = torch.view_as_complex(M.view(-1, 2)).reshape((4 * m + 1,) * d)
    b = torch.view_as_complex(b.view(-1, 2)).reshape(max(T, 1), -1)[:T]
    return (M, b, inf.as_dict()) if info else (M, b)


def solve_workspace_size(d: int, m: int, T: int, nlam: int, ctx: Optional[Context] = None) -> int:
    """Bytes of the workspace fk_solve needs (and in which it keeps the factors for the gradients)."""
    ctx = ctx or default_context(0)
    nb = C.c_size_t()
    _lib.check(ctx.lib.fk_solve_workspace_size(ctx.h, d, m, T, nlam, C.byref(nb)), "fk_solve_workspace_size")
    return nb.value


def solve(M: torch.Tensor, b: torch.Tensor, m: int, lambdas: Sequence[float], penalty: str = "sobolev",
          s: float = 1.0, ctx: Optional[Context] = None, info: bool = False, ws: Optional[torch.Tensor] = None,
          **pen_kw):
    """theta [nlam, T, N] complex128 from the generator M and right-hand sides b [T, N].

    ws: an explicit uint8 device workspace (at least solve_workspace_size bytes) that keeps the
    factors for heldout_mse / fit_backward; default: the context's cached workspace."""
    ctx = ctx or default_context(M.device.index or 0)
    ctx.bind_stream()
    d = M.dim()
    Mr = torch.view_as_real(M.contiguous()).contiguous()
    br = torch.view_as_real(b.contiguous()).contiguous()
    T = b.shape[0]
    lams = (C.c_double * len(lambdas))(*[float(v) for v in lambdas])
    nlam = len(lambdas)
    nb = C.c_size_t()
    _lib.check(ctx.lib.fk_solve_workspace_size(ctx.h, d, m, T, nlam, C.byref(nb)), "fk_solve_workspace_size")
    if ws is None:
        ws = ctx.workspace(nb.value)
    elif ws.numel() < nb.value:
        raise ValueError("workspace too small")
    nb = C.c_size_t(ws.numel())
    theta = torch.empty((nlam, T, _modes(m, d), 2), dtype=torch.float64, device=M.device)
    pen, keep = _penalty(penalty, s, **pen_kw)
    inf = fk_fit_info()
    _lib.check(ctx.lib.fk_solve(ctx.h, d, m, _ptr(Mr), T, _ptr(br), lams, nlam, C.byref(pen), _ptr(theta), _ptr(ws),
                                nb.value, C.byref(inf)), "fk_solve")
    del keep
    th = torch.view_as_complex(theta)
    return (th, inf.as_dict()) if info else th


def restrict(M: torch.Tensor, b: Optional[torch.Tensor], m_from: int, m_to: int, ctx: Optional[Context] = None):
    """(M, b) for the basis ||k||_inf <= m_to from those of m_from >= m_to (centred sub-blocks)."""
    ctx = ctx or default_context(M.device.index or 0)
    ctx.bind_stream()
    d = M.dim()
    Mr = torch.view_as_real(M.contiguous()).contiguous()
    T = 0 if b is None else b.shape[0]
    br = None if b is None else torch.view_as_real(b.contiguous()).contiguous()
    Mo = torch.empty(((4 * m_to + 1) ** d, 2), dtype=torch.float64, device=M.device)
    bo = torch.empty((max(T, 1), _modes(m_to, d), 2), dtype=torch.float64, device=M.device)
    _lib.check(ctx.lib.fk_restrict(ctx.h, d, m_from, m_to, T, _ptr(Mr), _ptr(br), _ptr(Mo), _ptr(bo)),
               "fk_restrict")
    Mo = torch.view_as_complex(Mo).reshape((4 * m_to + 1,) * d)
    return Mo, (None if b is None else torch.view_as_complex(bo)[:T])


def toeplitz_apply(M: torch.Tensor, x: torch.Tensor, m: int, ctx: Optional[Context] = None) -> torch.Tensor:
    """y = Sigma x for Sigma[k, l] = M[l - k] by FFT; x [V, N] complex128 on the device."""
    ctx = ctx or default_context(M.device.index or 0)
    ctx.bind_stream()
    d = M.dim()
    Mr = torch.view_as_real(M.contiguous()).contiguous()
    xr = torch.view_as_real(x.reshape(-1, _modes(m, d)).contiguous()).contiguous()
    V = xr.shape[0]
    nb = C.c_size_t()
    _lib.check(ctx.lib.fk_toeplitz_apply_workspace_size(ctx.h, d, m, V, C.byref(nb)),
               "fk_toeplitz_apply_workspace_size")
    ws = ctx.workspace(nb.value)
    y = torch.empty_like(xr)
    _lib.check(ctx.lib.fk_toeplitz_apply(ctx.h, d, m, _ptr(Mr), V, _ptr(xr), _ptr(y), _ptr(ws), nb.value),
               "fk_toeplitz_apply")
    return torch.view_as_complex(y).reshape(x.shape)


def solve_cg(M: torch.Tensor, b: torch.Tensor, m: int, lambdas: Sequence[float], penalty: str = "sobolev",
             s: float = 1.0, tol: float = 1e-10, maxit: int = 1000, ctx: Optional[Context] = None,
             info: bool = False, collocation=None, **pen_kw):
    """theta [nlam, T, N] complex128 by Jacobi-preconditioned conjugate gradients with FFT products.

    collocation = (mu, Mr, D) adds the physics term mu D^* Sigma_r D: Mr the generator of the
    collocation points (from gram(Xr, None, m)), D [N] complex128 the operator symbol, on the device.
    With info=True also returns {"iters": iterations of the slowest system,
    "relres": [nlam, T] final ||b - A theta|| / ||b||}."""
    ctx = ctx or default_context(M.device.index or 0)
    ctx.bind_stream()
    d = M.dim()
    Mr = torch.view_as_real(M.contiguous()).contiguous()
    br = torch.view_as_real(b.contiguous()).contiguous()
    T = b.shape[0]
    lams = (C.c_double * len(lambdas))(*[float(v) for v in lambdas])
    nlam = len(lambdas)
    nb = C.c_size_t()
    theta = torch.empty((nlam, T, _modes(m, d), 2), dtype=torch.float64, device=M.device)
    pen, keep = _penalty(penalty, s, **pen_kw)
    it = C.c_int()
    rel = (C.c_double * (nlam * T))()
    if collocation is None:
        _lib.check(ctx.lib.fk_solve_cg_workspace_size(ctx.h, d, m, T, nlam, C.byref(nb)),
                   "fk_solve_cg_workspace_size")
        ws = ctx.workspace(nb.value)
        _lib.check(ctx.lib.fk_solve_cg(ctx.h, d, m, _ptr(Mr), T, _ptr(br), lams, nlam, C.byref(pen), float(tol),
                                       int(maxit), _ptr(theta), C.byref(it), rel, _ptr(ws), nb.value),
                   "fk_solve_cg")
    else:
        mu, Mcol, Dsym = collocation
        Mcr = torch.view_as_real(Mcol.contiguous()).contiguous()
        Dr = torch.view_as_real(Dsym.reshape(-1).to(torch.complex128).contiguous()).contiguous()
        if Dr.shape[0] != _modes(m, d) or Mcr.numel() != Mr.numel():
            raise ValueError("collocation generator or symbol of the wrong size")
        _lib.check(ctx.lib.fk_solve_cg_collocation_workspace_size(ctx.h, d, m, T, nlam, C.byref(nb)),
                   "fk_solve_cg_collocation_workspace_size")
        ws = ctx.workspace(nb.value)
        _lib.check(ctx.lib.fk_solve_cg_collocation(ctx.h, d, m, _ptr(Mr), T, _ptr(br), lams, nlam, C.byref(pen),
                                                   float(mu), _ptr(Mcr), _ptr(Dr), float(tol), int(maxit),
                                                   _ptr(theta), C.byref(it), rel, _ptr(ws), nb.value),
                   "fk_solve_cg_collocation")
    del keep
    th = torch.view_as_complex(theta)
    if info:
        return th, {"iters": it.value, "relres": [[rel[l * T + t] for t in range(T)] for l in range(nlam)]}
    return th


def fit_kept_workspace_size(d: int, n: int, T: int, m: int, nlam: int, ctx: Optional[Context] = None):
    """(solve_bytes, scratch_bytes) of fk_fit_kept: the part that keeps the factors, and the type-1 scratch."""
    ctx = ctx or default_context(0)
    sb, tb = C.c_size_t(), C.c_size_t()
    _lib.check(ctx.lib.fk_fit_kept_workspace_size(ctx.h, d, n, T, m, nlam, C.byref(sb), C.byref(tb)),
               "fk_fit_kept_workspace_size")
    return sb.value, tb.value


def fit(X: torch.Tensor, Y: torch.Tensor, m: int, lambdas, penalty: str = "sobolev", s: float = 1.0,
        ctx: Optional[Context] = None, info: bool = False, ws: Optional[torch.Tensor] = None, **pen_kw):
    """fit(X, Y, m, lambda(s), penalty) -> theta [nlam, T, N] complex128 (the type-1 stage and the solve
    in one call).

    ws: an explicit uint8 device workspace (at least the solve_bytes of fit_kept_workspace_size) that
    keeps the factors for heldout_mse / fit_backward; the type-1 stage then runs in the context's
    cached workspace (fk_fit_kept).  Default: both in the context's cached workspace (fk_fit)."""
    ctx = ctx or default_context(X.device.index or 0)
    ctx.bind_stream()
    if isinstance(lambdas, (int, float)):
        lambdas = [float(lambdas)]
    X = _dev_tensor(X, "X")
    Y = _dev_tensor(Y, "Y")
    d, n = X.shape
    T = Y.shape[0]
    lams = (C.c_double * len(lambdas))(*[float(v) for v in lambdas])
    nlam = len(lambdas)
    theta = torch.empty((nlam, T, _modes(m, d), 2), dtype=torch.float64, device=X.device)
    pen, keep = _penalty(penalty, s, **pen_kw)
    inf = fk_fit_info()
    if ws is None:
        nb = C.c_size_t()
        _lib.check(ctx.lib.fk_fit_workspace_size(ctx.h, d, n, T, m, nlam, C.byref(nb)), "fk_fit_workspace_size")
        w = ctx.workspace(nb.value)
        _lib.check(ctx.lib.fk_fit(ctx.h, d, n, _dtype_code(X), _ptr(X), T, _ptr(Y), m, lams, nlam, C.byref(pen),
                                  _ptr(theta), _ptr(w), nb.value, C.byref(inf)), "fk_fit")
    else:
        if ws.device != X.device or ws.dtype != torch.uint8 or not ws.is_contiguous():
            raise ValueError("ws must be a contiguous uint8 tensor on the device of X")
        _, tb = fit_kept_workspace_size(d, n, T, m, nlam, ctx)
        w = ctx.workspace(tb)
        _lib.check(ctx.lib.fk_fit_kept(ctx.h, d, n, _dtype_code(X), _ptr(X), T, _ptr(Y), m, lams, nlam,
                                       C.byref(pen), _ptr(theta), _ptr(ws), ws.numel(), _ptr(w), tb,
                                       C.byref(inf)), "fk_fit_kept")
    del keep
    th = torch.view_as_complex(theta)
    return (th, inf.as_dict()) if info else th


def predict(theta: torch.Tensor, Xq: torch.Tensor, m: int, ctx: Optional[Context] = None) -> torch.Tensor:
    """f_theta(Xq) = Re sum_k theta_k exp(i k.x) by type-2 NUFFT; theta [T, N] complex128 -> [T, nq] float32."""
    ctx = ctx or default_context(Xq.device.index or 0)
    ctx.bind_stream()
    Xq = _dev_tensor(Xq, "Xq")
    d, nq = Xq.shape
    th = torch.view_as_real(theta.reshape(-1, _modes(m, d)).contiguous()).contiguous()
    T = th.shape[0]
    nb = C.c_size_t()
    _lib.check(ctx.lib.fk_predict_workspace_size(ctx.h, d, m, T, C.byref(nb)), "fk_predict_workspace_size")
    ws = ctx.workspace(nb.value)
    out = torch.empty((T, nq), dtype=torch.float32, device=Xq.device)
    _lib.check(ctx.lib.fk_predict(ctx.h, d, m, T, _ptr(th), nq, _dtype_code(Xq), _ptr(Xq), _ptr(out), _ptr(ws),
                                  nb.value), "fk_predict")
    return out


def predict_noalloc(theta: torch.Tensor, Xq: torch.Tensor, m: int, ctx: Optional[Context] = None) -> torch.Tensor:
    """predict() through fk_predict_noalloc: no workspace, the library's fixed device array instead.
    Calls on one device share that array and must not overlap."""
    ctx = ctx or default_context(Xq.device.index or 0)
    ctx.bind_stream()
    Xq = _dev_tensor(Xq, "Xq")
    d, nq = Xq.shape
    th = torch.view_as_real(theta.reshape(-1, _modes(m, d)).contiguous()).contiguous()
    T = th.shape[0]
    out = torch.empty((T, nq), dtype=torch.float32, device=Xq.device)
    _lib.check(ctx.lib.fk_predict_noalloc(ctx.h, d, m, T, _ptr(th), nq, _dtype_code(Xq), _ptr(Xq), _ptr(out)),
               "fk_predict_noalloc")
    return out


def heldout_mse(Mv: torch.Tensor, bv: torch.Tensor, yv2: torch.Tensor, m: int, nlam: int,
                ctx: Context, ws: Optional[torch.Tensor] = None) -> torch.Tensor:
    """mse [nlam, T] of the last solve kept in ws (default: ctx's workspace) against held-out statistics."""
    ctx.bind_stream()
    d = Mv.dim()
    T = bv.shape[0]
    Mr = torch.view_as_real(Mv.contiguous()).contiguous()
    br = torch.view_as_real(bv.contiguous()).contiguous()
    y2 = yv2.to(torch.float64).contiguous()
    out = torch.empty((nlam, T), dtype=torch.float64, device=Mv.device)
    ws = ctx._ws if ws is None else ws
    _lib.check(ctx.lib.fk_heldout_mse(ctx.h, d, m, T, nlam, _ptr(Mr), _ptr(br), _ptr(y2), _ptr(out), _ptr(ws),
                                      ws.numel()), "fk_heldout_mse")
    return out


def mean_square(Y: torch.Tensor, ctx: Optional[Context] = None) -> torch.Tensor:
    """[T] float64: mean of Y[t]**2 over the points (the constant term of the held-out MSE)."""
    ctx = ctx or default_context(Y.device.index or 0)
    ctx.bind_stream()
    Y = _dev_tensor(Y, "Y")
    Y2 = Y.reshape(-1, Y.shape[-1]) if Y.dim() > 1 else Y.reshape(1, -1)
    out = torch.empty(Y2.shape[0], dtype=torch.float64, device=Y.device)
    _lib.check(ctx.lib.fk_mean_square(ctx.h, Y2.shape[0], Y2.shape[1], _dtype_code(Y2), _ptr(Y2), _ptr(out)),
               "fk_mean_square")
    return out


def fit_backward(grad_mse: torch.Tensor, m: int, d: int, ctx: Context, want_theta: bool = False,
                 grad_theta_in: Optional[torch.Tensor] = None, ws: Optional[torch.Tensor] = None):
    """Gradients (log lambda [nlam], p [N], theta [nlam, T, N] or None) of
    Loss = sum(grad_mse * mse) + (the loss whose Wirtinger gradient dLoss/dconj(theta) is grad_theta_in),
    through theta = A^-1 b, with the factors kept in ws (default: ctx's workspace).  The theta gradient
    returned (want_theta) is the Wirtinger gradient of sum(grad_mse * mse) with theta held fixed."""
    ctx.bind_stream()
    nlam, T = grad_mse.shape
    g = grad_mse.to(torch.float64).contiguous()
    N = _modes(m, d)
    gl = torch.empty(nlam, dtype=torch.float64, device=g.device)
    gp = torch.empty(N, dtype=torch.float64, device=g.device)
    gt = torch.empty((nlam, T, N, 2), dtype=torch.float64, device=g.device) if want_theta else None
    gin = None
    if grad_theta_in is not None:
        gin = torch.view_as_real(grad_theta_in.to(torch.complex128).reshape(nlam, T, N).contiguous()).contiguous()
    ws = ctx._ws if ws is None else ws
    _lib.check(ctx.lib.fk_fit_backward(ctx.h, d, m, T, nlam, _ptr(g), _ptr(gin), _ptr(gl), _ptr(gp), _ptr(gt),
                                       _ptr(ws), ws.numel()), "fk_fit_backward")
    return gl, gp, (torch.view_as_complex(gt) if want_theta else None)


def additive_gram(X: torch.Tensor, Y: torch.Tensor, m: int, ctx: Optional[Context] = None):
    """Block Gram B [d(2m+1), d(2m+1)] and stacked b [T, d(2m+1)] of the additive model (Sec. 5)."""
    ctx = ctx or default_context(X.device.index or 0)
    ctx.bind_stream()
    X = _dev_tensor(X, "X")
    Y = _dev_tensor(Y, "Y")
    d, n = X.shape
    T = Y.shape[0]
    Nc = d * (2 * m + 1)
    nb = C.c_size_t()
    _lib.check(ctx.lib.fk_additive_gram_workspace_size(ctx.h, d, n, T, m, C.byref(nb)), "ws")
    ws = ctx.workspace(nb.value)
    B = torch.empty((Nc, Nc, 2), dtype=torch.float64, device=X.device)
    b = torch.empty((T, Nc, 2), dtype=torch.float64, device=X.device)
    inf = fk_fit_info()
    _lib.check(ctx.lib.fk_additive_gram(ctx.h, d, n, _dtype_code(X), _ptr(X), T, _ptr(Y), m, _ptr(B), _ptr(b),
                                        _ptr(ws), nb.value, C.byref(inf)), "fk_additive_gram")
    return torch.view_as_complex(B), torch.view_as_complex(b)


def additive_fit(X: torch.Tensor, Y: torch.Tensor, m: int, lambdas, s: float = 1.0, ctx: Optional[Context] = None,
                 info: bool = False):
    """theta [nlam, T, d(2m+1)] of the additive model with per-component Sobolev weights 1 + |k|^(2s)."""
    ctx = ctx or default_context(X.device.index or 0)
    ctx.bind_stream()
    if isinstance(lambdas, (int, float)):
        lambdas = [float(lambdas)]
    X = _dev_tensor(X, "X")
    Y = _dev_tensor(Y, "Y")
    d, n = X.shape
    T = Y.shape[0]
    lams = (C.c_double * len(lambdas))(*[float(v) for v in lambdas])
    nb = C.c_size_t()
    _lib.check(ctx.lib.fk_additive_fit_workspace_size(ctx.h, d, n, T, m, len(lambdas), C.byref(nb)), "ws")
    ws = ctx.workspace(nb.value)
    theta = torch.empty((len(lambdas), T, d * (2 * m + 1), 2), dtype=torch.float64, device=X.device)
    inf = fk_fit_info()
    _lib.check(ctx.lib.fk_additive_fit(ctx.h, d, n, _dtype_code(X), _ptr(X), T, _ptr(Y), m, lams, len(lambdas),
                                       float(s), _ptr(theta), _ptr(ws), nb.value, C.byref(inf)), "fk_additive_fit")
    th = torch.view_as_complex(theta)
    return (th, inf.as_dict()) if info else th


def autotune_table() -> str:
    """The library's table of measured launch shapes, one "<key> = <knob>=<value> ... ms=<t>" per line."""
    lib = _lib.load()
    n = C.c_size_t()
    _lib.check(lib.fk_autotune_table(None, 0, C.byref(n)), "fk_autotune_table")
    buf = C.create_string_buffer(n.value + 1)
    _lib.check(lib.fk_autotune_table(buf, n.value + 1, C.byref(n)), "fk_autotune_table")
    return buf.value.decode()


def autotune_load(path: str) -> None:
    """Merge a table file (lines "<key> = <knob>=<int> ...") into the library's table."""
    _lib.check(_lib.load().fk_autotune_load(path.encode()), "fk_autotune_load")


def autotune_clear() -> None:
    _lib.check(_lib.load().fk_autotune_clear(), "fk_autotune_clear")


def generate_uniform(seed: int, d: int, n: int, lo=None, hi=None, start: int = 0, device: int = 0,
                     ctx: Optional[Context] = None) -> torch.Tensor:
    """Philox4x32-10 uniform points [d, n] float32 on the device (same stream as the test generator)."""
    ctx = ctx or default_context(device)
    ctx.bind_stream()
    lo = [-math.pi] * d if lo is None else list(lo)
    hi = [math.pi] * d if hi is None else list(hi)
    X = torch.empty((d, n), dtype=torch.float32, device=f"cuda:{device}")
    clo = (C.c_double * d)(*lo)
    chi = (C.c_double * d)(*hi)
    _lib.check(ctx.lib.fk_generate_uniform(ctx.h, seed, d, n, start, clo, chi, _ptr(X)), "fk_generate_uniform")
    return X


def generate_targets(seed: int, X: torch.Tensor, ntgt: int, sigma: float = 0.1, start: int = 0,
                     ctx: Optional[Context] = None) -> torch.Tensor:
    """Y_t = sin(t x1) cos(x2) + sigma N(0,1), t = 1..ntgt, float32 [ntgt, n] on the device."""
    ctx = ctx or default_context(X.device.index or 0)
    ctx.bind_stream()
    n = X.shape[1]
    Y = torch.empty((ntgt, n), dtype=torch.float32, device=X.device)
    _lib.check(ctx.lib.fk_generate_targets(ctx.h, seed, ntgt, n, start, _ptr(X), float(sigma), _ptr(Y)),
               "fk_generate_targets")
    return Y


class KernelRidgeGridLoss(torch.autograd.Function):
    """Held-out MSE of the fitted estimator over a grid of lambdas and targets.

    forward(loglam [nlam] float64, p [N] float64, X, Y, Xv, Yv, m)
        -> (mse [nlam, T] float64, theta [nlam, T, N] complex128)
    The fit uses the diagonal penalty p (e.g. Sobolev weights).  Both outputs are differentiable:
    backward runs one adjoint solve per (lambda, target) with the kept factors, on the combined
    right-hand side of the mse term and of any other use of theta, and returns the gradients with
    respect to log lambda and p.  Each apply keeps its factors in a workspace of its own, so several
    applies (cross-validation folds, repeated calls) can be alive in one graph.  The held-out Gram is
    computed on a second host thread, in a second library context on a second stream of the device,
    while the fit runs; applies on one device are therefore not to be issued from several threads at
    once.  Not in the paper: it makes the lambda grid search of Sec. 5 differentiable.
    """

    @staticmethod
    def forward(ctx_, loglam, p, X, Y, Xv, Yv, m):
        fkc = default_context(X.device.index or 0)
        lams = torch.exp(loglam.detach()).cpu().tolist()
        d = X.shape[0]
        # The fit (type-1 stage in the context's shared workspace, factors in this apply's own), and
        # meanwhile the held-out Gram on a second host thread, in a second context on a stream of
        # its own (the library calls release the interpreter lock): its kernels fill the GPU around
        # the fit's instead of following them.
        sb, _ = fit_kept_workspace_size(d, X.shape[1], Y.shape[0], m, len(lams), fkc)
        kept = torch.empty(sb, dtype=torch.uint8, device=X.device)
        vctx = _validation_context(fkc)
        main = torch.cuda.current_stream(X.device)
        vs = _validation_stream(X.device)
        vs.wait_stream(main)
        held: dict = {}

        def _heldout():
            try:
                with torch.cuda.stream(vs):
                    held["Mv"], held["bv"] = gram(Xv, Yv, m, ctx=vctx)
                    held["yv2"] = mean_square(Yv, vctx)
            except BaseException as e:   # re-raised on the calling thread
                held["err"] = e

        # The first apply of a held-out shape runs its Gram after the fit instead, so that the
        # launch-shape tuner (which times candidates on the call's own data) times it alone.
        key = (X.device.index, tuple(Xv.shape), tuple(Yv.shape), Xv.dtype, m)
        if key in _heldout_seen:
            worker = threading.Thread(target=_heldout)
            worker.start()
            try:
                theta = fit(X, Y, m, lams, penalty="diag", p=p.detach(), ctx=fkc, ws=kept)
            finally:
                worker.join()
        else:
            theta = fit(X, Y, m, lams, penalty="diag", p=p.detach(), ctx=fkc, ws=kept)
            vs.wait_stream(main)
            _heldout()
            _heldout_seen.add(key)
        if "err" in held:
            raise held["err"]
        main.wait_stream(vs)
        Mv, bv, yv2 = held["Mv"], held["bv"], held["yv2"]
        for t in (Mv, bv, yv2):
            t.record_stream(main)
        mse = heldout_mse(Mv, bv, yv2, m, len(lams), fkc, ws=kept)
        ctx_.fkc = fkc
        ctx_.kept = kept
        ctx_.m = m
        ctx_.d = d
        ctx_.set_materialize_grads(False)
        return mse, theta

    @staticmethod
    def backward(ctx_, grad_mse, grad_theta):
        if grad_mse is None:
            nlam, T = grad_theta.shape[:2]
            grad_mse = torch.zeros((nlam, T), dtype=torch.float64, device=grad_theta.device)
        # PyTorch's gradient of a complex tensor is 2 dLoss/dconj(theta); the library takes dLoss/dconj(theta)
        gin = None if grad_theta is None else 0.5 * grad_theta
        gl, gp, _ = fit_backward(grad_mse.contiguous(), ctx_.m, ctx_.d, ctx_.fkc, grad_theta_in=gin, ws=ctx_.kept)
        return gl, gp, None, None, None, None, None


_valctx: dict = {}
_valstream: dict = {}
_heldout_seen: set = set()


def _validation_stream(device) -> torch.cuda.Stream:
    """The held-out Gram's stream on this device (default priority, created once)."""
    dev = torch.device(device)
    s = _valstream.get(dev.index)
    if s is None:
        s = torch.cuda.Stream(device=dev)
        _valstream[dev.index] = s
    return s


def _validation_context(fkc: Context) -> Context:
    """A second context (own workspace) so the held-out Gram does not overwrite the fit's workspace."""
    c = _valctx.get(fkc.device)
    if c is None:
        c = Context(fkc.device)
        _valctx[fkc.device] = c
    return c
