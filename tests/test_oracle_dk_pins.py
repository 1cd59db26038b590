"""Pins of the oracle's general derivatives of K (oracle_logdk_batch), each
integrand over its own peak and interval (Section 4.1, Eq. (13)).

Independent of the oracle's own formulas:

* closed forms at half-integer order: K_{1/2}(x) = sqrt(pi/2) x^{-1/2} e^{-x}
  and K_{3/2}(x) = sqrt(pi/2) (x^{-1/2} + x^{-3/2}) e^{-x} (DLMF 10.39.2 and
  the order recurrence), differentiated b times in x by Leibniz' rule;
* the order derivative at v = 1/2, sqrt(pi/(2x)) E1(2x) e^{x} (DLMF 10.38.7),
  with E1 from scipy;
* the order recurrence K_{v+1} - K_{v-1} = (2v/x) K_v (DLMF 10.29.1)
  differentiated a times in v:
      D_a(v+1) - D_a(v-1) = (2a/x) D_{a-1}(v) + (2v/x) D_a(v),
  which ties every order in v to the one below it;
* the derivative recurrence dK_v/dx = -(K_{v-1} + K_{v+1})/2 (DLMF 10.29.1)
  differentiated a times in v and b times in x, which ties order b + 1 in x to
  order b at the neighbouring orders;
* the modified Bessel equation x^2 K'' + x K' - (x^2 + v^2) K = 0 (DLMF 10.25.1)
  and its derivative in v;
* signs, evenness in v, and the exact zero of odd v-derivatives at v = 0;
* agreement with the companion-integral first and second derivatives of log K
  (oracle_logk_hess_batch), which integrate over f's interval instead;
* mpmath's besselk differentiated numerically in v and x at 30 digits.
"""

from math import comb

import numpy as np
import pytest
from scipy.special import exp1

import oracle

X = np.geomspace(0.02, 60.0, 23)


def D(v, x, a, b):
    """Signed d^a/dv^a d^b/dx^b K_v(x) from the oracle."""
    lg, s = oracle.logdk(v, x, a, b)
    return s * np.exp(lg)


def _leibniz(p_terms, x, b):
    """d^b/dx^b of sqrt(pi/2) sum_p x^{-p} e^{-x}: (-1)^b sqrt(pi/2) e^{-x}
    sum_p sum_k C(b, k) (p)_k x^{-p-k}, with (p)_k the rising factorial."""
    total = np.zeros_like(x)
    for p in p_terms:
        for k in range(b + 1):
            rising = np.prod([p + j for j in range(k)]) if k else 1.0
            total += comb(b, k) * rising * x ** (-p - k)
    return (-1.0) ** b * np.sqrt(np.pi / 2) * np.exp(-x) * total


@pytest.mark.parametrize("b", range(6))
def test_half_order_x_derivatives(b):
    for v, p_terms in ((0.5, (0.5,)), (-0.5, (0.5,)), (1.5, (0.5, 1.5))):
        ref = _leibniz(p_terms, X, b)
        lg, s = oracle.logdk(np.full_like(X, v), X, 0, b)
        assert np.all(s == (-1.0) ** b)
        err = np.abs(lg - np.log(np.abs(ref))) / np.maximum(1.0, np.abs(np.log(np.abs(ref))))
        assert err.max() <= 2e-15, (v, b, err.max())


def test_order_derivative_at_half():
    x = np.geomspace(0.02, 20.0, 19)
    ref = np.sqrt(np.pi / (2 * x)) * exp1(2 * x) * np.exp(x)
    for v, sgn in ((0.5, 1.0), (-0.5, -1.0)):
        lg, s = oracle.logdk(np.full_like(x, v), x, 1, 0)
        assert np.all(s == sgn)
        np.testing.assert_allclose(np.exp(lg), ref, rtol=1e-14, atol=0)


@pytest.mark.parametrize("a", [1, 2, 3, 4])
def test_order_recurrence_in_v(a):
    # (mixed orders are tied to these through the x recurrence below)
    v = np.array([0.3, 0.5, 1.0, 1.7, 2.5, 4.0, 7.5])
    vv, xx = (q.ravel() for q in np.meshgrid(v, X, indexing="ij"))
    lhs = D(vv + 1, xx, a, 0) - D(vv - 1, xx, a, 0)
    t1 = (2 * a / xx) * D(vv, xx, a - 1, 0)
    t2 = (2 * vv / xx) * D(vv, xx, a, 0)
    scale = np.abs(D(vv + 1, xx, a, 0)) + np.abs(D(vv - 1, xx, a, 0)) + np.abs(t1) + np.abs(t2)
    assert (np.abs(lhs - t1 - t2) / scale).max() <= 1e-14


@pytest.mark.parametrize("a", [0, 1, 2, 3])
@pytest.mark.parametrize("b", [0, 1, 2, 3])
def test_x_recurrence(a, b):
    v = np.array([0.0, 0.3, 0.5, 1.0, 2.5, 6.0])
    vv, xx = (q.ravel() for q in np.meshgrid(v, X, indexing="ij"))
    lhs = D(vv, xx, a, b + 1)
    lo, hi = D(vv - 1, xx, a, b), D(vv + 1, xx, a, b)
    rhs = -0.5 * (lo + hi)
    scale = np.abs(lhs) + 0.5 * (np.abs(lo) + np.abs(hi))
    ok = scale > 0  # odd a at v = 0: every term is zero
    assert (np.abs(lhs - rhs)[ok] / scale[ok]).max() <= 1e-14
    assert np.all(lhs[~ok] == 0.0)


def test_bessel_equation_and_its_v_derivative():
    v = np.array([0.0, 0.4, 1.0, 2.5, 6.0, 15.0])
    vv, xx = (q.ravel() for q in np.meshgrid(v, X, indexing="ij"))
    K, K1, K2 = (D(vv, xx, 0, b) for b in range(3))
    terms = np.stack([xx ** 2 * K2, xx * K1, (xx ** 2 + vv ** 2) * K])
    res = xx ** 2 * K2 + xx * K1 - (xx ** 2 + vv ** 2) * K
    assert (np.abs(res) / np.abs(terms).sum(axis=0)).max() <= 1e-14
    # d/dv: x^2 dK''/dv + x dK'/dv - (x^2 + v^2) dK/dv - 2 v K = 0
    Kv, Kv1, Kv2 = (D(vv, xx, 1, b) for b in range(3))
    terms = np.stack([xx ** 2 * Kv2, xx * Kv1, (xx ** 2 + vv ** 2) * Kv, 2 * vv * K])
    res = xx ** 2 * Kv2 + xx * Kv1 - (xx ** 2 + vv ** 2) * Kv - 2 * vv * K
    s = np.abs(terms).sum(axis=0)
    ok = s > 0
    assert (np.abs(res)[ok] / s[ok]).max() <= 1e-14


def test_signs_symmetry_and_zeros():
    x = np.array([0.1, 1.0, 10.0])
    for a in range(5):
        for b in range(4):
            lp, sp = oracle.logdk(np.full(3, 1.3), x, a, b)
            lm, sm = oracle.logdk(np.full(3, -1.3), x, a, b)
            assert np.array_equal(lp, lm)
            assert np.all(sp == (-1.0) ** b)
            assert np.all(sm == (-1.0) ** b * (-1.0) ** a)
            l0, s0 = oracle.logdk(np.zeros(3), x, a, b)
            if a % 2:
                assert np.all(l0 == -np.inf) and np.all(s0 == 0.0)
            else:
                assert np.all(np.isfinite(l0)) and np.all(s0 == (-1.0) ** b)
    # conventions away from the domain
    lg, s = oracle.logdk(np.array([np.nan, 1.0, 1.0, 1.0, np.inf]), np.array([1.0, -1.0, 0.0, np.inf, 1.0]), 1, 1)
    assert np.isnan(lg[0]) and np.isnan(lg[1]) and np.isnan(s[0]) and np.isnan(s[1])
    assert lg[2] == np.inf and lg[3] == -np.inf and lg[4] == np.inf


def test_matches_companion_integrals():
    v = np.array([0.0, 0.5, 1.3, 4.0, 12.0, 40.0])
    vv, xx = (q.ravel() for q in np.meshgrid(v, np.geomspace(1e-2, 1e2, 9), indexing="ij"))
    H = oracle.logk_hess(vv, xx)
    lk = H[:, 0]
    assert np.max(np.abs(oracle.logdk(vv, xx, 0, 0)[0] - lk) / np.maximum(1, np.abs(lk))) <= 1e-15

    def check(a, b, ref_ratio, tol):
        # compare log |D_ab| with log K + log |D_ab / K| from the companion
        # integrals, in the mixed measure used for log K (the outputs are
        # logs of magnitude up to ~200, so a ratio formed from them would
        # carry their FP64 rounding)
        lg, s = oracle.logdk(vv, xx, a, b)
        nz = ref_ratio != 0
        assert np.all(np.sign(ref_ratio[nz]) == s[nz])
        assert np.all(lg[~nz] == -np.inf)
        ref = lk[nz] + np.log(np.abs(ref_ratio[nz]))
        assert np.max(np.abs(lg[nz] - ref) / np.maximum(1.0, np.abs(ref))) <= tol, (a, b)

    check(1, 0, H[:, 1], 1e-14)
    check(0, 1, H[:, 2], 1e-14)
    # K''/K = d2 log K + (d log K)^2
    check(2, 0, H[:, 3] + H[:, 1] ** 2, 1e-14)
    check(0, 2, H[:, 4] + H[:, 2] ** 2, 1e-14)
    check(1, 1, H[:, 5] + H[:, 1] * H[:, 2], 1e-14)


def test_mpmath_derivatives():
    # a library routine at 30 digits: mpmath's besselk differentiated
    # numerically in v and x (mp.diff), at stratified points and orders <= 3
    import mpmath as mp
    mp.mp.dps = 30
    pts = [(0.3, 0.05), (1.3, 0.7), (4.5, 2.0), (12.0, 30.0), (25.0, 3.0), (-2.2, 9.0)]
    for a, b in [(1, 0), (0, 1), (2, 0), (1, 1), (0, 3), (3, 1), (2, 2)]:
        v = np.array([p[0] for p in pts])
        x = np.array([p[1] for p in pts])
        lg, s = oracle.logdk(v, x, a, b)
        for i, (vi, xi) in enumerate(pts):
            ref = mp.diff(lambda vv, xx: mp.besselk(vv, xx), (mp.mpf(vi), mp.mpf(xi)), (a, b))
            got = s[i] * mp.exp(lg[i])
            assert abs(got - ref) <= 1e-13 * abs(ref), (a, b, vi, xi, float(got), float(ref))
