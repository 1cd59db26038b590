"""ctypes binding of libbessel.so (the C ABI in include/bessel.h).

Argument marshalling only: every step of the computation runs in the HIP
kernels behind the C ABI.  There is no CPU fallback; a missing library raises.
"""

from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libbessel.so")

F32 = 0
F64 = 1
RANGE_NEWTON = 0
RANGE_MLP = 1
RANGE_MLP_TABLE = 2

STATUS = {
    0: "BESSEL_OK",
    -1: "BESSEL_ERR_ARG",
    -2: "BESSEL_ERR_DTYPE",
    -3: "BESSEL_ERR_NBINS",
    -4: "BESSEL_ERR_RANGE_MODE",
    -5: "BESSEL_ERR_HIP",
    -6: "BESSEL_ERR_ALIAS",
    -7: "BESSEL_ERR_UNSUPPORTED",
    -8: "BESSEL_ERR_ORDER",
}

# Every symbol include/bessel.h declares, with its ctypes signature.
_vp = ctypes.c_void_p
_i64 = ctypes.c_int64
_int = ctypes.c_int
SIGNATURES = {
    "bessel_logk": (_int, [_int, _i64, _vp, _vp, _vp, _int, _int, _vp, _vp]),
    "bessel_logk_dv_dx": (_int, [_int, _i64, _vp, _vp, _vp, _vp, _vp, _vp, _int, _int, _vp, _vp]),
    "bessel_range": (_int, [_int, _i64, _vp, _vp, _vp, _vp, _vp, _vp, _int, _vp, _vp, _vp]),
    "bessel_logk_backward": (_int, [_int, _i64, _vp, _vp, _vp, _vp, _vp, _vp]),
    "bessel_logk_hess": (_int, [_int, _i64, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _int, _vp]),
    "bessel_hess_vjp": (_int, [_int, _i64, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp]),
    "bessel_logdk": (_int, [_int, _i64, _vp, _vp, _int, _int, _vp, _vp, _int, _vp]),
    "bessel_set_split_threshold": (_int, [_i64, _vp]),
    "bessel_mlp_create": (_int, [_vp, _i64, _vp]),
    "bessel_mlp_destroy": (_int, [_vp]),
    "bessel_mlp_set_params": (_int, [_vp, _vp, _i64]),
    "bessel_mlp_get_params": (_int, [_vp, _vp, _i64]),
    "bessel_mlp_train": (_int, [_vp, _vp, _i64, _vp, _vp, _vp, _vp]),
    "bessel_mlp_loss_grad": (_int, [_vp, _i64, _vp, _vp, _vp, _vp, ctypes.c_float, _vp, _vp, _vp]),
    "bessel_mlp_forward": (_int, [_vp, _i64, _vp, _vp, _vp, _int, _vp]),
    "bessel_mlp_adam_step": (_int, [_vp, _vp, ctypes.c_float, ctypes.c_float, ctypes.c_float, ctypes.c_float, _vp]),
    "bessel_mlp_fallback_count": (_int, [_vp, _vp]),
    "bessel_gh_logk_sum": (_int, [_i64, _vp, _vp, _vp, _vp, _i64, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _int, _int,
                                  _vp, _vp]),
    "bessel_gh_logk_sum_noalloc": (_int, [_i64, _vp, _vp, _vp, _vp, _i64, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _int,
                                          _int, _vp, _vp]),
    "bessel_last_error": (ctypes.c_char_p, []),
    "bessel_version": (ctypes.c_char_p, []),
}

_lib = None


class BesselError(RuntimeError):
    """A non-zero status from the C ABI."""


def load(path: str | None = None):
    """Load libbessel.so (built in-tree by ``paper_2108_11560_amd.build``)."""
    global _lib
    if _lib is not None and path is None:
        return _lib
    p = path or LIB_PATH
    if not os.path.exists(p):
        raise ImportError(
            f"{p} is missing: build it with `python -m paper_2108_11560_amd.build` "
            "(the GPU path has no CPU fallback)"
        )
    lib = ctypes.CDLL(p)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    if path is None:
        _lib = lib
    return lib


def check(rc: int, what: str) -> None:
    if rc != 0:
        msg = load().bessel_last_error().decode(errors="replace")
        raise BesselError(f"{what} failed: {STATUS.get(rc, rc)}: {msg}")
