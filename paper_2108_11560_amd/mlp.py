"""Learned bracket predictor: Python handle over the C ABI (bessel_mlp_*).

The predictor maps (log v, log x) to the integration bracket [t0, t1] of the
method (Section 2.1, Eq. (7)-(8)); it is trained on the brackets the Newton
range finder produces, and every predicted bracket is checked by the fused
kernel, with the Newton path as fallback.  See include/bessel.h for the
network, the parameter layout and the check.

All arithmetic runs in the library's kernels; this module marshals arguments,
owns the handle, initialises weights, and searches the two output margins.
"""

from __future__ import annotations

import ctypes
import os

import numpy as np
import torch

from . import _lib
from ._lib import check, load

NWEIGHTS = 4482
NPARAMS = 4490
HIDDEN = 64
# offsets in the parameter vector
O_META = 4482
DEFAULT_NORM = (1.0, 3.0, 0.0, 4.0)  # m_v, s_v, m_x, s_x: z ~ [-2.6, 1] x [-1.7, 1.7] on v < 50, 1e-3 < x < 1e3


class TrainCfg(ctypes.Structure):
    _fields_ = [
        ("steps", ctypes.c_int64),
        ("batch", ctypes.c_int64),
        ("lr", ctypes.c_float),
        ("lr_final", ctypes.c_float),
        ("beta1", ctypes.c_float),
        ("beta2", ctypes.c_float),
        ("adam_eps", ctypes.c_float),
        ("alpha", ctypes.c_float),
        ("seed", ctypes.c_uint64),
    ]


def _vp(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p(0)


def _stream(dev):
    return ctypes.c_void_p(torch.cuda.current_stream(dev).cuda_stream)


def glorot_params(seed: int = 0, norm=DEFAULT_NORM, margins=(0.0, 0.0)) -> np.ndarray:
    """Glorot-uniform weights, zero biases, the given normalisation and margins."""
    rng = np.random.default_rng(seed)

    def u(fan_out, fan_in):
        a = np.sqrt(6.0 / (fan_in + fan_out))
        return rng.uniform(-a, a, size=(fan_out, fan_in))

    p = np.concatenate([
        u(HIDDEN, 2).ravel(), np.zeros(HIDDEN),
        u(HIDDEN, HIDDEN).ravel(), np.zeros(HIDDEN),
        u(2, HIDDEN).ravel(), np.zeros(2),
        np.array([norm[0], norm[1], norm[2], norm[3], margins[0], margins[1], 0.0, 0.0]),
    ]).astype(np.float32)
    assert p.size == NPARAMS
    return p


class RangeMLP:
    """A bessel_mlp handle on the current device."""

    def __init__(self, params: np.ndarray | None = None):
        lib = load()
        self._lib = lib
        h = ctypes.c_void_p()
        arr = None
        if params is not None:
            arr = np.ascontiguousarray(params, dtype=np.float32)
            if arr.size != NPARAMS:
                raise ValueError(f"expected {NPARAMS} parameters")
        ptr = arr.ctypes.data_as(ctypes.POINTER(ctypes.c_float)) if arr is not None else None
        check(lib.bessel_mlp_create(ptr, NPARAMS, ctypes.byref(h)), "bessel_mlp_create")
        self._h = h

    @property
    def handle(self) -> int:
        return self._h.value

    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            self._lib.bessel_mlp_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # parameters ----------------------------------------------------------
    def params(self) -> np.ndarray:
        out = np.empty(NPARAMS, dtype=np.float32)
        check(self._lib.bessel_mlp_get_params(self._h, out.ctypes.data_as(ctypes.POINTER(ctypes.c_float)), NPARAMS),
              "bessel_mlp_get_params")
        return out

    def set_params(self, p: np.ndarray):
        arr = np.ascontiguousarray(p, dtype=np.float32)
        if arr.size != NPARAMS:
            raise ValueError(f"expected {NPARAMS} parameters")
        check(self._lib.bessel_mlp_set_params(self._h, arr.ctypes.data_as(ctypes.POINTER(ctypes.c_float)), NPARAMS),
              "bessel_mlp_set_params")

    def set_margins(self, margin_t1: float, margin_t0: float):
        p = self.params()
        p[O_META + 4] = margin_t1
        p[O_META + 5] = margin_t0
        self.set_params(p)

    def save(self, path: str):
        np.save(path, self.params())

    @classmethod
    def load_file(cls, path: str) -> "RangeMLP":
        return cls(np.load(path, allow_pickle=False))

    # training ------------------------------------------------------------
    def train(self, v: torch.Tensor, x: torch.Tensor, steps: int = 2000, batch: int = 8192, lr: float = 3e-3,
              lr_final: float = 1e-4, alpha: float = 4.0, seed: int = 0, beta1: float = 0.9,
              beta2: float = 0.999, adam_eps: float = 1e-8) -> np.ndarray:
        """Train on FP32 device inputs; returns the per-step losses."""
        if v.dtype != torch.float32 or x.dtype != torch.float32 or v.device.type != "cuda":
            raise TypeError("training inputs must be float32 CUDA tensors")
        v, x = v.contiguous(), x.contiguous()
        cfg = TrainCfg(steps, batch, lr, lr_final, beta1, beta2, adam_eps, alpha, seed)
        losses = np.empty(max(steps, 1), dtype=np.float32)
        with torch.cuda.device(v.device):
            rc = self._lib.bessel_mlp_train(self._h, ctypes.byref(cfg), v.numel(), _vp(v), _vp(x),
                                            losses.ctypes.data_as(ctypes.POINTER(ctypes.c_float)), _stream(v.device))
        check(rc, "bessel_mlp_train")
        return losses[:steps]

    def loss_grad(self, v, x, t0, t1, alpha: float = 4.0):
        loss = torch.empty(1, dtype=torch.float32, device=v.device)
        grad = torch.empty(NWEIGHTS, dtype=torch.float32, device=v.device)
        with torch.cuda.device(v.device):
            rc = self._lib.bessel_mlp_loss_grad(self._h, v.numel(), _vp(v), _vp(x), _vp(t0), _vp(t1),
                                                ctypes.c_float(alpha), _vp(loss), _vp(grad), _stream(v.device))
        check(rc, "bessel_mlp_loss_grad")
        return loss, grad

    def adam_step(self, grad: torch.Tensor, lr: float, beta1: float = 0.9, beta2: float = 0.999,
                  eps: float = 1e-8):
        with torch.cuda.device(grad.device):
            rc = self._lib.bessel_mlp_adam_step(self._h, _vp(grad.contiguous()), ctypes.c_float(lr),
                                                ctypes.c_float(beta1), ctypes.c_float(beta2), ctypes.c_float(eps),
                                                _stream(grad.device))
        check(rc, "bessel_mlp_adam_step")

    def forward(self, v, x, mode: int = 1) -> torch.Tensor:
        y = torch.empty((v.numel(), 2), dtype=torch.float32, device=v.device)
        with torch.cuda.device(v.device):
            rc = self._lib.bessel_mlp_forward(self._h, v.numel(), _vp(v), _vp(x), _vp(y), int(mode),
                                              _stream(v.device))
        check(rc, "bessel_mlp_forward")
        return y

    def fallback_count(self) -> int:
        c = ctypes.c_int()
        check(self._lib.bessel_mlp_fallback_count(self._h, ctypes.byref(c)), "bessel_mlp_fallback_count")
        return c.value


def calibrate_margins(mlp: RangeMLP, v: torch.Tensor, x: torch.Tensor, target_fallback: float = 0.005,
                      grid_t1=(0.0, 0.01, 0.02, 0.04, 0.07, 0.1, 0.15, 0.2, 0.3),
                      grid_t0=(0.0, 0.01, 0.02, 0.04, 0.07, 0.1), range: str = "mlp"):
    """Smallest (margin_t1, margin_t0) on the grid whose fallback rate on (v, x)
    is at most target_fallback (by the library's own check, in the learned
    range mode ``range``: "mlp" or "mlp_table"); returns (margin_t1, margin_t0, rate)."""
    from . import bessel_range
    best = None
    for m1 in grid_t1:
        for m0 in grid_t0:
            mlp.set_margins(m1, m0)
            *_, fb = bessel_range(v, x, range=range, mlp=mlp, want_fallback=True)
            rate = float(fb.float().mean())
            if rate <= target_fallback:
                if best is None or m1 + m0 < best[0] + best[1]:
                    best = (m1, m0, rate)
                break
    if best is None:
        m1, m0 = grid_t1[-1], grid_t0[-1]
        mlp.set_margins(m1, m0)
        *_, fb = bessel_range(v, x, range=range, mlp=mlp, want_fallback=True)
        best = (m1, m0, float(fb.float().mean()))
    mlp.set_margins(best[0], best[1])
    return best
