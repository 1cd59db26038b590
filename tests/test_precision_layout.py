"""Why the FP32 path forms the per-node argument in FP64 (CPU, numpy).

On the curve K_v(x) = 1 (log K = 0, so the mixed error is the absolute error
of log K) the node argument log cosh(v t) - x cosh t - g(t_p) subtracts
terms of size ~v t_p.  A 128-bin trapezoid over the exact FP32-margin bracket
with FP32 exponentials is evaluated twice: with the argument in FP32
arithmetic (every operation rounded to FP32) and with it in FP64.  The first
misses the FP32 bar of 1e-5 from v ~ 200 on (terms ~ 250); the second stays
far below it at every order up to 1000.  The reference is the oracle.
"""

import numpy as np

import oracle

F32 = np.float32
LOG_EPS32_MARGIN = -15.9423851528787422 - 1.0


def on_unit_curve(v):
    """x with log K_v(x) = 0, by bisection on the oracle."""
    lo, hi = 1e-3, 2.0 * v
    for _ in range(70):
        mid = np.sqrt(lo * hi)
        if oracle.logk(np.array([v]), np.array([mid]))[0] > 0:
            lo = mid
        else:
            hi = mid
    return np.sqrt(lo * hi)


def log_cosh64(z):
    z = np.abs(z)
    return z + np.log1p(np.exp(-2 * z)) - np.log(2.0)


def trapezoid(v, x, t0, t1, G, fp32_argument, nbins=128):
    h = (t1 - t0) / nbins
    t = t0 + h * np.arange(nbins + 1)
    c = np.ones(nbins + 1)
    c[0] = c[-1] = 0.5
    if fp32_argument:
        tf, vf, xf, Gf = t.astype(F32), F32(v), F32(x), F32(G)
        vt = vf * tf
        lc = vt + np.log1p(np.exp(F32(-2) * vt)) - F32(np.log(2.0))
        a = (lc - xf * np.cosh(tf)) - Gf
    else:
        a = log_cosh64(v * t) - x * np.cosh(t) - G
    w = np.exp(np.asarray(a, dtype=F32)).astype(np.float64)  # FP32 exponential in both
    return G + np.log(h * np.sum(c * w))


def test_fp64_argument_needed_for_large_orders():
    vs = np.array([10.0, 50.0, 200.0, 500.0, 1000.0])
    xs = np.array([on_unit_curve(v) for v in vs])
    _, G, t0, t1 = oracle.range_exact(vs, xs, LOG_EPS32_MARGIN)
    ref = oracle.logk(vs, xs)
    assert np.all(np.abs(ref) < 1e-10)
    e32 = np.array([abs(trapezoid(vs[i], xs[i], t0[i], t1[i], G[i], True) - ref[i]) for i in range(vs.size)])
    e64 = np.array([abs(trapezoid(vs[i], xs[i], t0[i], t1[i], G[i], False) - ref[i]) for i in range(vs.size)])
    print("FP32 argument", e32, "FP64 argument", e64)
    assert np.all(e64 <= 1e-6)
    assert e32[-2] > 1e-5 and e32[-1] > 1e-5
