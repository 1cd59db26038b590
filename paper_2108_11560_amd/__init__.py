"""Batched log K_v(x) and its derivatives on MI355X (gfx950) HIP kernels.

Takekawa, "Fast parallel calculation of modified Bessel function of the second
kind and its derivatives" (arXiv 2108.11560): K_v(x) as the integral of
cosh(v t) exp(-x cosh t) over t >= 0 (Section 2, Eq. (1)-(2)), evaluated per
element by locating the peak of the log-integrand, bracketing the range where
it lies within log eps of the peak, and summing a fixed number of trapezoid
bins in log space (Sections 2.1-2.4); derivatives in v and x from the
companion integrals of Section 4.1, Eq. (13), over the same bins.

This module marshals torch tensors (device memory, the current HIP stream) into
the C ABI of ``libbessel.so`` (``include/bessel.h``); every step of the
computation runs in the library's kernels.

    logk(v, x, nbins=128)                  -> log K_v(x)
    logk_dv_dx(v, x, grad_out=None, ...)   -> (log K, d/dv log K, d/dx log K)
    logk_hess(v, x)                        -> (log K, d/dv, d/dx, d2/dv2, d2/dx2, d2/dvdx)
    logdk(v, x, a, b)                      -> (log |d^a/dv^a d^b/dx^b K|, its sign), each
                                              integrand over its own peak and bracket
    bessel_range(v, x)                     -> (t0, t1, t_p, g(t_p))
    log_bessel_k(v, x)                     -> log K with autograd (BesselLogK),
                                              twice differentiable on the Newton bracket
"""

from __future__ import annotations

import contextlib
import ctypes

import torch

from . import _lib
from ._lib import F32, F64, RANGE_MLP, RANGE_MLP_TABLE, RANGE_NEWTON, BesselError, check, load  # noqa: F401

__all__ = [
    "logk",
    "logk_dv_dx",
    "logk_hess",
    "logdk",
    "set_split_threshold",
    "bessel_range",
    "log_bessel_k",
    "gh_logk_sum",
    "BesselLogK",
    "BesselError",
    "load",
]


def _dtype_code(t: torch.Tensor) -> int:
    if t.dtype == torch.float32:
        return F32
    if t.dtype == torch.float64:
        return F64
    raise TypeError(f"dtype {t.dtype} not supported (float32 or float64)")


def _stream_ptr(device: torch.device):
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def _check_pair(v: torch.Tensor, x: torch.Tensor):
    if not (isinstance(v, torch.Tensor) and isinstance(x, torch.Tensor)):
        raise TypeError("v and x must be torch tensors")
    if v.device.type != "cuda" or x.device.type != "cuda":
        raise ValueError("v and x must be on a GPU device (the library has no CPU path)")
    if v.device != x.device:
        raise ValueError("v and x must be on the same device")
    if v.dtype != x.dtype:
        raise TypeError("v and x must have the same dtype")
    if v.shape != x.shape:
        raise ValueError(f"shape mismatch {tuple(v.shape)} vs {tuple(x.shape)}")
    return v.contiguous(), x.contiguous()


def _on(device: torch.device):
    """The device context for a call, skipped when it is already current (a
    per-call cost that dominates small batches)."""
    if device.index is None or device.index == torch.cuda.current_device():
        return contextlib.nullcontext()
    return torch.cuda.device(device)


def _ptr(t: torch.Tensor | None):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p(0)


def _mlp_ptr(mlp):
    if mlp is None:
        return ctypes.c_void_p(0)
    return ctypes.c_void_p(mlp.handle)


def _range_code(range_: str) -> int:
    if range_ == "newton":
        return RANGE_NEWTON
    if range_ == "mlp":
        return RANGE_MLP
    if range_ == "mlp_table":
        return RANGE_MLP_TABLE
    raise ValueError(f"range must be 'newton', 'mlp' or 'mlp_table', not {range_!r}")


def logk(v: torch.Tensor, x: torch.Tensor, nbins: int = 128, range: str = "newton", mlp=None) -> torch.Tensor:
    """log K_v(x) elementwise (no autograd; see :func:`log_bessel_k`)."""
    v, x = _check_pair(v, x)
    out = torch.empty_like(v)
    lib = load()
    with _on(v.device):
        rc = lib.bessel_logk(_dtype_code(v), v.numel(), _ptr(v), _ptr(x), _ptr(out), int(nbins),
                             _range_code(range), _mlp_ptr(mlp), _stream_ptr(v.device))
    check(rc, "bessel_logk")
    return out


def logk_dv_dx(v: torch.Tensor, x: torch.Tensor, grad_out: torch.Tensor | None = None, nbins: int = 128,
               range: str = "newton", mlp=None, want_logk: bool = True):
    """(log K, d/dv log K, d/dx log K); the derivatives are multiplied by grad_out if given."""
    v, x = _check_pair(v, x)
    if grad_out is not None:
        if grad_out.shape != v.shape or grad_out.dtype != v.dtype or grad_out.device != v.device:
            raise ValueError("grad_out must match v in shape, dtype and device")
        grad_out = grad_out.contiguous()
    lk = torch.empty_like(v) if want_logk else None
    dv = torch.empty_like(v)
    dx = torch.empty_like(v)
    lib = load()
    with _on(v.device):
        rc = lib.bessel_logk_dv_dx(_dtype_code(v), v.numel(), _ptr(v), _ptr(x), _ptr(grad_out), _ptr(lk), _ptr(dv),
                                   _ptr(dx), int(nbins), _range_code(range), _mlp_ptr(mlp), _stream_ptr(v.device))
    check(rc, "bessel_logk_dv_dx")
    return lk, dv, dx


def logk_hess(v: torch.Tensor, x: torch.Tensor, nbins: int = 128, want=(True,) * 6):
    """(log K, d/dv, d/dx, d2/dv2, d2/dx2, d2/dvdx) of log K from one pass
    (Newton bracket); an output whose ``want`` flag is False comes back None."""
    v, x = _check_pair(v, x)
    outs = [torch.empty_like(v) if w else None for w in want]
    lib = load()
    with _on(v.device):
        rc = lib.bessel_logk_hess(_dtype_code(v), v.numel(), _ptr(v), _ptr(x), *(_ptr(o) for o in outs), int(nbins),
                                  _stream_ptr(v.device))
    check(rc, "bessel_logk_hess")
    return tuple(outs)


def logdk(v: torch.Tensor, x: torch.Tensor, order_v: int, order_x: int, nbins: int = 128, want_sign: bool = True):
    """(log |D|, sign of D) for D = d^order_v/dv^order_v d^order_x/dx^order_x K_v(x),
    each derivative integrand over its own peak and bracket (Section 4.1,
    Eq. (13)); the sign comes back None when ``want_sign`` is False."""
    v, x = _check_pair(v, x)
    out = torch.empty_like(v)
    sgn = torch.empty_like(v) if want_sign else None
    lib = load()
    with _on(v.device):
        rc = lib.bessel_logdk(_dtype_code(v), v.numel(), _ptr(v), _ptr(x), int(order_v), int(order_x), _ptr(out),
                              _ptr(sgn), int(nbins), _stream_ptr(v.device))
    check(rc, "bessel_logdk")
    return out, sgn


def set_split_threshold(n: int) -> int:
    """Batches of at most n elements use the 16-lanes-per-element kernels
    (latency of small batches); returns the previous threshold."""
    prev = ctypes.c_int64()
    check(load().bessel_set_split_threshold(int(n), ctypes.byref(prev)), "bessel_set_split_threshold")
    return prev.value


def bessel_range(v: torch.Tensor, x: torch.Tensor, range: str = "newton", mlp=None, want_fallback: bool = False):
    """Integration range (t0, t1), peak t_p and g(t_p) per element (and the fallback flags)."""
    v, x = _check_pair(v, x)
    t0, t1, tp, gp = torch.empty_like(v), torch.empty_like(v), torch.empty_like(v), torch.empty_like(v)
    fb = torch.empty(v.shape, dtype=torch.uint8, device=v.device) if want_fallback else None
    lib = load()
    with _on(v.device):
        rc = lib.bessel_range(_dtype_code(v), v.numel(), _ptr(v), _ptr(x), _ptr(t0), _ptr(t1), _ptr(tp), _ptr(gp),
                              _range_code(range), _mlp_ptr(mlp), _ptr(fb), _stream_ptr(v.device))
    check(rc, "bessel_range")
    return (t0, t1, tp, gp, fb) if want_fallback else (t0, t1, tp, gp)


def gh_logk_sum(lam: torch.Tensor, alpha: torch.Tensor, delta: torch.Tensor, mu: torch.Tensor, y: torch.Tensor,
                grad_sum: torch.Tensor | None = None, nbins: int = 128, want_grad: bool = True,
                no_alloc: bool = False, range: str = "newton", mlp=None):
    """Per-set sums of log K_{lam-1/2}(alpha sqrt(delta^2 + (y - mu)^2)) over the shared
    samples y, and (optionally) their gradients in (lam, alpha, delta, mu), FP32.
    ``range``: "newton" or "mlp_table" (the predictor ``mlp`` read from its
    table, checked per element, Newton bracket where the check fails).
    ``no_alloc`` calls ``bessel_gh_logk_sum_noalloc`` (partials in the library's
    static device array; calls on one GPU must not overlap)."""
    sets = [t.contiguous() for t in (lam, alpha, delta, mu)]
    y = y.contiguous()
    for t in (*sets, y) + ((grad_sum,) if grad_sum is not None else ()):
        if t.dtype != torch.float32 or t.device.type != "cuda":
            raise TypeError("gh_logk_sum takes float32 CUDA tensors")
    n = sets[0].numel()
    if any(t.numel() != n for t in sets) or (grad_sum is not None and grad_sum.numel() != n):
        raise ValueError("lam, alpha, delta, mu (and grad_sum) must have the same length")
    dev = y.device
    out = torch.empty(n, dtype=torch.float32, device=dev)
    grads = ([torch.empty(n, dtype=torch.float32, device=dev) for _ in (0, 1, 2, 3)] if want_grad
             else [None] * 4)
    gs = grad_sum.contiguous() if grad_sum is not None else None
    lib = load()
    with _on(dev):
        fn = lib.bessel_gh_logk_sum_noalloc if no_alloc else lib.bessel_gh_logk_sum
        rc = fn(n, *(_ptr(t) for t in sets), y.numel(), _ptr(y), _ptr(gs), _ptr(out), *(_ptr(g) for g in grads),
                int(nbins), _range_code(range), _mlp_ptr(mlp), _stream_ptr(dev))
    check(rc, "bessel_gh_logk_sum_noalloc" if no_alloc else "bessel_gh_logk_sum")
    return (out, *grads) if want_grad else out


class _BesselDLogK(torch.autograd.Function):
    """(d/dv log K, d/dx log K) as a differentiable function of (v, x): the
    forward runs ``bessel_logk_hess`` (first and second derivatives from one
    pass), the backward ``bessel_hess_vjp`` with the saved second derivatives."""

    @staticmethod
    def forward(ctx, v, x, nbins):
        _, dv, dx, dvv, dxx, dvx = logk_hess(v, x, nbins=nbins, want=(False, True, True, True, True, True))
        ctx.save_for_backward(dvv, dxx, dvx)
        return dv, dx

    @staticmethod
    @torch.autograd.function.once_differentiable
    def backward(ctx, g_dv, g_dx):
        dvv, dxx, dvx = ctx.saved_tensors
        g_dv = g_dv.contiguous() if g_dv is not None else None
        g_dx = g_dx.contiguous() if g_dx is not None else None
        gv = torch.empty_like(dvv) if ctx.needs_input_grad[0] else None
        gx = torch.empty_like(dvv) if ctx.needs_input_grad[1] else None
        if gv is None and gx is None:
            return None, None, None
        if g_dv is None and g_dx is None:
            return (torch.zeros_like(dvv) if gv is not None else None,
                    torch.zeros_like(dvv) if gx is not None else None, None)
        lib = load()
        with _on(dvv.device):
            rc = lib.bessel_hess_vjp(_dtype_code(dvv), dvv.numel(), _ptr(g_dv), _ptr(g_dx), _ptr(dvv), _ptr(dxx),
                                     _ptr(dvx), _ptr(gv), _ptr(gx), _stream_ptr(dvv.device))
        check(rc, "bessel_hess_vjp")
        return gv, gx, None


class BesselLogK(torch.autograd.Function):
    """log K_v(x) with a hand-written backward.

    The forward runs the fused kernel that also produces d/dv and d/dx of log K
    from the same bins whenever an input needs a gradient; backward multiplies
    the saved derivatives by the upstream gradient in the library's
    ``bessel_logk_backward`` kernel.  Under ``create_graph`` (second-order
    differentiation, Newton bracket only) the backward instead builds its
    result from :class:`_BesselDLogK`, whose own backward uses the second
    derivatives of the same bins.
    """

    @staticmethod
    def forward(ctx, v, x, nbins=128, range="newton", mlp=None):
        ctx.nbins, ctx.range = nbins, range
        if ctx.needs_input_grad[0] or ctx.needs_input_grad[1]:
            lk, dv, dx = logk_dv_dx(v, x, None, nbins=nbins, range=range, mlp=mlp)
            ctx.save_for_backward(v, x, dv, dx)
            return lk
        return logk(v, x, nbins=nbins, range=range, mlp=mlp)

    @staticmethod
    def backward(ctx, go):
        v, x, dv, dx = ctx.saved_tensors
        if torch.is_grad_enabled():
            if ctx.range != "newton":
                raise BesselError("second-order differentiation needs the Newton bracket")
            dvt, dxt = _BesselDLogK.apply(v, x, ctx.nbins)
            gv = go * dvt if ctx.needs_input_grad[0] else None
            gx = go * dxt if ctx.needs_input_grad[1] else None
            return gv, gx, None, None, None
        go = go.contiguous()
        gv = torch.empty_like(dv) if ctx.needs_input_grad[0] else None
        gx = torch.empty_like(dx) if ctx.needs_input_grad[1] else None
        lib = load()
        with _on(dv.device):
            rc = lib.bessel_logk_backward(_dtype_code(dv), dv.numel(), _ptr(go), _ptr(dv), _ptr(dx), _ptr(gv),
                                          _ptr(gx), _stream_ptr(dv.device))
        check(rc, "bessel_logk_backward")
        return gv, gx, None, None, None


def log_bessel_k(v: torch.Tensor, x: torch.Tensor, nbins: int = 128, range: str = "newton", mlp=None):
    """log K_v(x) with autograd support in v and x (second order on the Newton bracket)."""
    if v.shape != x.shape:
        v, x = torch.broadcast_tensors(v, x)
    return BesselLogK.apply(v, x, nbins, range, mlp)
