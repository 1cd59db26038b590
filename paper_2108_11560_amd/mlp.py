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
import hashlib
import json
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


# What a checkpoint's parameter vector means: the network's shape and
# activations, the order of the parameter vector and its metadata slots.  A
# file written for another layout is refused.
LAYOUT = ("2-64-64-2; h1 = clamp(W1 z + b1, -1, 1); h2 = u(3 - u^2)/2, u = clamp((W2 h1 + b2)/1.5, -1, 1); "
          "y = W3 h2 + b3; params W1(64x2) b1 W2(64x64) b2 W3(2x64) b3, then m_v s_v m_x s_x margin_t1 margin_t0 0 0")
CHECKPOINT_VERSION = 1


def write_checkpoint(path: str, params: np.ndarray, provenance: dict | None) -> None:
    """Parameters plus a JSON record (layout, version, provenance) in one .npz,
    readable without unpickling."""
    arr = np.ascontiguousarray(params, dtype=np.float32)
    if arr.size != NPARAMS:
        raise ValueError(f"expected {NPARAMS} parameters")
    meta = {"layout": LAYOUT, "version": CHECKPOINT_VERSION, "nparams": NPARAMS,
            "params_sha256": hashlib.sha256(arr.tobytes()).hexdigest(), "provenance": provenance or {}}
    with open(path, "wb") as fh:  # the exact path, whatever its suffix
        np.savez(fh, params=arr, meta=np.array(json.dumps(meta, sort_keys=True)))


def read_checkpoint(path: str):
    """(params, provenance) of a file write_checkpoint wrote; raises ValueError
    for another layout or version, a wrong size, or parameters that do not
    match their recorded hash."""
    f = np.load(path, allow_pickle=False)
    if not isinstance(f, np.lib.npyio.NpzFile):
        raise ValueError(f"{path}: not a predictor checkpoint (no layout record)")
    with f:
        if "meta" not in f or "params" not in f:
            raise ValueError(f"{path}: not a predictor checkpoint (no layout record)")
        meta = json.loads(str(f["meta"]))
        params = np.asarray(f["params"], dtype=np.float32)
    if meta.get("layout") != LAYOUT or meta.get("version") != CHECKPOINT_VERSION:
        raise ValueError(f"{path}: written for another network layout or format version")
    if params.size != NPARAMS or meta.get("nparams") != NPARAMS:
        raise ValueError(f"{path}: expected {NPARAMS} parameters, found {params.size}")
    if hashlib.sha256(params.tobytes()).hexdigest() != meta.get("params_sha256"):
        raise ValueError(f"{path}: parameters do not match their recorded hash")
    return params, meta["provenance"]


def _sha256_of(*tensors) -> str:
    h = hashlib.sha256()
    for t in tensors:
        h.update(np.ascontiguousarray(t.detach().cpu().numpy()).tobytes())
    return h.hexdigest()


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
        # how the parameters came about: training run, labels, margins
        self.provenance: dict = {}

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
        # as stored: FP32 parameters
        self.provenance["margins"] = {"t1": float(np.float32(margin_t1)), "t0": float(np.float32(margin_t0))}

    def save(self, path: str):
        """Parameters with the layout record and the provenance (training
        configuration and seed, hashes of the training inputs and of their
        Newton labels, margins and their calibration) in one .npz file."""
        write_checkpoint(path, self.params(), self.provenance)

    @classmethod
    def load_file(cls, path: str) -> "RangeMLP":
        params, prov = read_checkpoint(path)
        net = cls(params)
        net.provenance = prov
        return net

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
        # the labels are the Newton brackets of the inputs at the FP32 eps,
        # which bessel_range returns bit for bit
        from . import bessel_range
        t0, t1, _, _ = bessel_range(v, x)
        self.provenance = {
            "train": {"steps": int(steps), "batch": int(batch), "lr": float(lr), "lr_final": float(lr_final),
                      "alpha": float(alpha), "seed": int(seed), "beta1": float(beta1), "beta2": float(beta2),
                      "adam_eps": float(adam_eps), "final_loss": float(losses[steps - 1]) if steps > 0 else None},
            "inputs": {"n": int(v.numel()), "sha256_v_x": _sha256_of(v, x)},
            "labels": {"kind": "Newton bracket, FP32 eps", "sha256_t0_t1": _sha256_of(t0, t1)},
            "library": self._lib.bessel_version().decode(errors="replace"),
        }
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


def calibrate_margins(mlp: RangeMLP, v: torch.Tensor, x: torch.Tensor, target_fallback: float = 0.001,
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
    mlp.provenance["calibration"] = {"target_fallback": float(target_fallback), "range": range,
                                     "n": int(v.numel()), "sha256_v_x": _sha256_of(v, x),
                                     "fallback_rate": best[2]}
    return best
