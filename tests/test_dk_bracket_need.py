"""Why derivatives of high order need brackets of their own (Section 4.1,
Eq. (13)): the 128-bin trapezoid of a derivative integrand taken over f's
bracket, the layout of the companion sums, stays at FP64 accuracy for orders
<= 2 but not for high orders in x, whose integrand t^a cosh^b(t) C(vt)
e^{-x cosh t} puts mass beyond f's interval.  Reference: the oracle's
adaptive quadrature over the integrand's own interval.  (The GPU path for
those orders, bessel_logdk, brackets each integrand itself; its parity is in
tests/test_logdk_gpu.py.)"""

import numpy as np
from scipy.special import logsumexp

import oracle
import workloads

LOG_EPS64 = -36.0436533891171560 - 1.0


def trapezoid_over_f_bracket(v, x, a, b, nbins=128):
    _, _, t0, t1 = oracle.range_exact(v, x, LOG_EPS64)
    out = np.empty(v.size)
    for i in range(v.size):
        t = np.linspace(t0[i], t1[i], nbins + 1)
        h = (t1[i] - t0[i]) / nbins
        vt = v[i] * t
        with np.errstate(divide="ignore"):  # log sinh(0) = -inf for odd a
            lc = vt + np.log1p(-np.exp(-2 * vt)) if a % 2 else vt + np.log1p(np.exp(-2 * vt))
        lt = a * np.log(np.where(t > 0, t, 1.0)) if a else 0.0
        lg = lt + b * (t + np.log1p(np.exp(-2 * t))) + lc - x[i] * np.cosh(t) - (b + 1) * np.log(2.0)
        if a:
            lg = np.where(t > 0, lg, -np.inf)
        w = np.full(t.size, h)
        w[0] = w[-1] = 0.5 * h
        out[i] = logsumexp(lg, b=w)
    return out


def test_low_orders_fit_f_bracket_high_orders_do_not():
    v, x, _ = workloads.scale_pairs(200, seed=47)
    err = {}
    for a, b in [(1, 0), (0, 1), (2, 0), (0, 2), (1, 1), (0, 8)]:
        ref, _ = oracle.logdk(v, x, a, b)
        got = trapezoid_over_f_bracket(v, x, a, b)
        err[(a, b)] = np.max(np.abs(got - ref) / np.maximum(1.0, np.abs(ref)))
    for k in [(1, 0), (0, 1), (2, 0), (0, 2), (1, 1)]:
        assert err[k] <= 1e-13, (k, err[k])
    # above the FP64 bar of 1e-12
    assert err[(0, 8)] > 1e-12, err[(0, 8)]
    print({k: float(e) for k, e in err.items()})
