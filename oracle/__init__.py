"""CPU oracle for log K_v(x) and its derivatives (test infrastructure only).

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  It shares no code with the GPU library
``paper_2108_11560_amd`` and never imports it.

The numerical work lives in ``oracle.c`` (x87 long double); this module builds
it with gcc and wraps its entry points with ctypes over numpy float64 arrays.

Entry points (all vectorised over float64 arrays of equal length):

* :func:`logk` -- the plain definition of Section 2, Eq. (1)-(2): log of the
  integral of cosh(v t) exp(-x cosh t) over t >= 0, by adaptive Gauss-Legendre
  quadrature; optionally d/dv and d/dx of log K from the companion integrals
  of Section 4.1, Eq. (13).
* :func:`range_exact` -- the exact peak of g and the truncation interval of
  Section 2.1, Eq. (7)-(8), by bisection.
* :func:`method_logk` -- Algorithms 1-3 with the trapezoid of Eq. (int), in the
  paper's order (readings documented in ``oracle.c``).
* :func:`trapezoid_brute` -- a single-element plain trapezoid with a huge bin
  count, used only to pin the adaptive rule.
* :func:`logdk` -- log |d^a/dv^a d^b/dx^b K_v(x)| and its sign for any orders
  (Section 4.1, Eq. (13)), each integrand over its own peak and interval.
"""

from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

_lib = None


def build(force: bool = True) -> str:
    """Compile ``oracle.c`` into ``liboracle.so`` with gcc (no fast-math)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(
            ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-Wall", "-o", tmp, _SRC, "-lm", "-lpthread"]
        )
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=True)
        lib = ctypes.CDLL(_LIB)
        dp = ctypes.POINTER(ctypes.c_double)
        lib.oracle_logk_batch.argtypes = [ctypes.c_int64, dp, dp, dp, dp, dp, ctypes.c_int]
        lib.oracle_logk_batch.restype = ctypes.c_int
        lib.oracle_logk_hess_batch.argtypes = [ctypes.c_int64, dp, dp, dp, ctypes.c_int]
        lib.oracle_logk_hess_batch.restype = ctypes.c_int
        lib.oracle_range_exact.argtypes = [ctypes.c_int64, dp, dp, ctypes.c_double, dp, dp, dp, dp, ctypes.c_int]
        lib.oracle_range_exact.restype = ctypes.c_int
        lib.oracle_method_batch.argtypes = [
            ctypes.c_int64, dp, dp, ctypes.c_int, ctypes.c_double, ctypes.c_int, ctypes.c_double,
            ctypes.c_int, dp, dp, dp, dp, ctypes.c_int,
        ]
        lib.oracle_method_batch.restype = ctypes.c_int
        lib.oracle_trapezoid_brute.argtypes = [
            ctypes.c_double, ctypes.c_double, ctypes.c_double, ctypes.c_double, ctypes.c_int64, dp,
        ]
        lib.oracle_trapezoid_brute.restype = ctypes.c_int
        lib.oracle_logdk_batch.argtypes = [ctypes.c_int64, dp, dp, ctypes.c_int, ctypes.c_int, dp, dp, ctypes.c_int]
        lib.oracle_logdk_batch.restype = ctypes.c_int
        _lib = lib
    return _lib


def default_threads() -> int:
    try:
        return max(1, len(os.sched_getaffinity(0)))
    except AttributeError:  # pragma: no cover
        return max(1, os.cpu_count() or 1)


def _arr(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64).ravel())


def _ptr(a: np.ndarray | None):
    if a is None:
        return ctypes.POINTER(ctypes.c_double)()
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def logk(v, x, deriv: bool = False, nthreads: int | None = None):
    """log K_v(x); with ``deriv`` also (d/dv log K, d/dx log K)."""
    lib = _load()
    v = _arr(v)
    x = _arr(x)
    if v.shape != x.shape:
        v, x = np.broadcast_arrays(v, x)
        v, x = _arr(v), _arr(x)
    n = v.size
    out = np.empty(n)
    dv = np.empty(n) if deriv else None
    dx = np.empty(n) if deriv else None
    rc = lib.oracle_logk_batch(n, _ptr(v), _ptr(x), _ptr(out), _ptr(dv), _ptr(dx), nthreads or default_threads())
    if rc != 0:
        raise ValueError("oracle_logk_batch rejected its arguments")
    return (out, dv, dx) if deriv else out


def logk_hess(v, x, nthreads: int | None = None):
    """log K_v(x) with its first and second derivatives: an (n, 6) array of
    log K, d/dv, d/dx, d2/dv2, d2/dx2, d2/dvdx of log K."""
    lib = _load()
    v, x = np.broadcast_arrays(_arr(v), _arr(x))
    v, x = _arr(v), _arr(x)
    n = v.size
    out = np.empty((n, 6))
    rc = lib.oracle_logk_hess_batch(n, _ptr(v), _ptr(x), _ptr(out), nthreads or default_threads())
    if rc != 0:
        raise ValueError("oracle_logk_hess_batch rejected its arguments")
    return out


def range_exact(v, x, log_eps: float, nthreads: int | None = None):
    """Exact (t_p, G, t0, t1) with [t0, t1] = {t : g(t) >= g(t_p) + log_eps}."""
    lib = _load()
    v, x = np.broadcast_arrays(_arr(v), _arr(x))
    v, x = _arr(v), _arr(x)
    n = v.size
    tp, G, t0, t1 = (np.empty(n) for _ in range(4))
    rc = lib.oracle_range_exact(n, _ptr(v), _ptr(x), float(log_eps), _ptr(tp), _ptr(G), _ptr(t0), _ptr(t1),
                                nthreads or default_threads())
    if rc != 0:
        raise ValueError("oracle_range_exact rejected its arguments")
    return tp, G, t0, t1


def method_logk(v, x, nbins: int = 128, log_eps: float = float(np.log(np.finfo(np.float64).eps)),
                halve_ok: bool = True, tol: float = 1.0, max_iter: int = 10, nthreads: int | None = None):
    """The paper's Algorithm 3 with Eq. (int); returns (logk, t_p, t0, t1)."""
    lib = _load()
    v, x = np.broadcast_arrays(_arr(v), _arr(x))
    v, x = _arr(v), _arr(x)
    n = v.size
    out, tp, t0, t1 = (np.empty(n) for _ in range(4))
    rc = lib.oracle_method_batch(n, _ptr(v), _ptr(x), int(nbins), float(log_eps), int(bool(halve_ok)),
                                 float(tol), int(max_iter), _ptr(out), _ptr(tp), _ptr(t0), _ptr(t1),
                                 nthreads or default_threads())
    if rc != 0:
        raise ValueError("oracle_method_batch rejected its arguments")
    return out, tp, t0, t1


def trapezoid_brute(v: float, x: float, lo: float, hi: float, nbins: int):
    """Plain trapezoid with ``nbins`` bins on [lo, hi]: (log K, d/dv log K, d/dx log K)."""
    lib = _load()
    out = np.empty(3)
    rc = lib.oracle_trapezoid_brute(float(v), float(x), float(lo), float(hi), int(nbins), _ptr(out))
    if rc != 0:
        raise ValueError("oracle_trapezoid_brute rejected its arguments")
    return out


def logdk(v, x, order_v: int, order_x: int, nthreads: int | None = None):
    """(log |D|, sign D) for D = d^order_v/dv^order_v d^order_x/dx^order_x K_v(x)
    (Section 4.1, Eq. (13)); sign is (-1)^order_x, times sign(v) for odd
    order_v, and 0 where D is exactly zero (odd order_v at v = 0)."""
    lib = _load()
    v, x = np.broadcast_arrays(_arr(v), _arr(x))
    v, x = _arr(v), _arr(x)
    n = v.size
    out, sign = np.empty(n), np.empty(n)
    rc = lib.oracle_logdk_batch(n, _ptr(v), _ptr(x), int(order_v), int(order_x), _ptr(out), _ptr(sign),
                                nthreads or default_threads())
    if rc != 0:
        raise ValueError("oracle_logdk_batch rejected its arguments")
    return out, sign
