"""Pins of the CPU oracle against facts that do not come from the oracle itself.

Each test fixes one part of the oracle with a closed form, an identity, a
library routine, an asymptotic expansion with its error bound, or a brute-force
sum.  A dropped term, a wrong sign or a wrong index in the integrands, the peak,
the truncation interval or the derivative integrals fails at least one of them:

* the integrand of Eq. (1)-(2)      -> closed forms at v = 1/2, 3/2; mpmath; scipy K0/K1;
                                      order recurrence; Hankel bound; small-x limits;
                                      the uniform large-order expansion (v to 1e5)
* d/dx (Section 4.1, Eq. (13))      -> recurrence identity for K'_v; closed forms at 1/2, 3/2
* d/dv (Section 4.1, Eq. (13))      -> DLMF 10.38.7 at v = 1/2; v = 0; oddness; mpmath diff;
                                      Richardson differences of log K
* truncation interval (Eq. (7)-(8)) -> its defining inequalities, evaluated in numpy
* adaptive rule                     -> a 2^16-bin brute-force trapezoid
* Algorithms 1-3 and Eq. (int)      -> agreement with the plain definition
"""

import math

import mpmath as mp
import numpy as np
import pytest
from scipy import special

import oracle
import workloads

LOG_EPS64 = float(np.log(np.finfo(np.float64).eps))


def mixed_err(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return np.abs(a - b) / np.maximum(1.0, np.abs(b))


XS = np.logspace(-3, 3, 61)


def test_half_order_closed_form():
    # K_{1/2}(x) = sqrt(pi / (2x)) e^{-x}  (DLMF 10.39.2; the p_0 = 1 case of Eq. (kvp)).
    ref = 0.5 * np.log(np.pi / (2 * XS)) - XS
    assert mixed_err(oracle.logk(np.full_like(XS, 0.5), XS), ref).max() <= 4e-16


def test_three_halves_closed_form():
    # K_{3/2}(x) = sqrt(pi / (2x)) e^{-x} (1 + 1/x): Eq. (recu) at u = 1/2 with K_{-1/2} = K_{1/2}.
    ref = 0.5 * np.log(np.pi / (2 * XS)) - XS + np.log1p(1.0 / XS)
    assert mixed_err(oracle.logk(np.full_like(XS, 1.5), XS), ref).max() <= 4e-16


def test_dx_closed_forms():
    # d/dx log K_{1/2} = -1/(2x) - 1 ; d/dx log K_{3/2} = -1/(2x) - 1 - 1/(x^2 + x).
    _, _, dx = oracle.logk(np.full_like(XS, 0.5), XS, deriv=True)
    ref = -0.5 / XS - 1.0
    assert (np.abs(dx - ref) / np.abs(ref)).max() <= 4e-16
    _, _, dx = oracle.logk(np.full_like(XS, 1.5), XS, deriv=True)
    ref = -0.5 / XS - 1.0 - 1.0 / (XS * XS + XS)
    assert (np.abs(dx - ref) / np.abs(ref)).max() <= 4e-16


def test_dv_half_order_dlmf_10_38_7():
    # dK_v/dv at v = 1/2 is sqrt(pi/(2x)) E1(2x) e^{x}, so d/dv log K = E1(2x) e^{2x}.
    x = np.logspace(-3, np.log10(300.0), 40)
    _, dv, _ = oracle.logk(np.full_like(x, 0.5), x, deriv=True)
    ref = special.exp1(2 * x) * np.exp(2 * x)
    assert (np.abs(dv - ref) / np.abs(ref)).max() <= 1e-14


def test_dv_zero_order_and_oddness():
    x = np.logspace(-3, 3, 25)
    _, dv0, _ = oracle.logk(np.zeros_like(x), x, deriv=True)
    assert np.all(dv0 == 0.0)
    v = np.linspace(0.1, 40.0, 25)
    lp, dvp, dxp = oracle.logk(v, x, deriv=True)
    lm, dvm, dxm = oracle.logk(-v, x, deriv=True)
    assert np.array_equal(lp, lm)  # K_{-v} = K_v (integrand even in v)
    assert np.array_equal(dvp, -dvm)
    assert np.array_equal(dxp, dxm)
    assert np.all(dvp > 0.0)  # K_v increases with v > 0


def test_order_recurrence():
    # K_{v+1} = K_{v-1} + (2v/x) K_v (Eq. (recu)), checked in log space.
    rng = np.random.default_rng(101)
    v = rng.uniform(1.0, 49.0, 400)
    x = 10.0 ** rng.uniform(-3, 3, 400)
    lm, l0, lp = oracle.logk(v - 1, x), oracle.logk(v, x), oracle.logk(v + 1, x)
    rhs = np.logaddexp(lm, np.log(2 * v / x) + l0)
    assert mixed_err(lp, rhs).max() <= 1e-15


def test_dx_recurrence_identity():
    # K'_v = -(K_{v-1} + K_{v+1}) / 2 (DLMF 10.29.2), and the paper's Eq. (deriv) with
    # log on the left: d/dx log K_v = -v/x - K_{v-1}/K_v.
    rng = np.random.default_rng(102)
    v = rng.uniform(0.0, 49.0, 400)
    x = 10.0 ** rng.uniform(-3, 3, 400)
    l0, _, dx = oracle.logk(v, x, deriv=True)
    lm = oracle.logk(np.abs(v - 1), x)
    lp = oracle.logk(v + 1, x)
    ref = -0.5 * (np.exp(lm - l0) + np.exp(lp - l0))
    # exp of a difference of rounded logs carries ~eps * |log K| relative error
    tol = 4e-16 * (4.0 + np.abs(l0) + np.abs(lm) + np.abs(lp))
    assert np.all(np.abs(dx - ref) / np.abs(ref) <= tol)
    ref2 = -v / x - np.exp(lm - l0)
    assert np.all(np.abs(dx - ref2) <= tol * (np.abs(ref) + v / x))


def test_dv_richardson():
    # Fourth-order central differences of the oracle's own log K in v.
    rng = np.random.default_rng(103)
    v = rng.uniform(0.5, 45.0, 60)
    x = 10.0 ** rng.uniform(-2, 2.5, 60)
    h = 2e-3
    f = lambda s: oracle.logk(s, x)  # noqa: E731
    fd = (-f(v + 2 * h) + 8 * f(v + h) - 8 * f(v - h) + f(v - 2 * h)) / (12 * h)
    _, dv, _ = oracle.logk(v, x, deriv=True)
    assert (np.abs(dv - fd) / np.maximum(1.0, np.abs(dv))).max() <= 1e-9


def test_integer_orders_scipy():
    x = np.logspace(-3, 3, 61)
    assert mixed_err(oracle.logk(np.zeros_like(x), x), np.log(special.k0e(x)) - x).max() <= 1e-15
    assert mixed_err(oracle.logk(np.ones_like(x), x), np.log(special.k1e(x)) - x).max() <= 1e-15


def _spot_points(n, seed):
    v, x, s = workloads.scale_pairs(4096, seed=seed)
    idx = workloads.stratified_subset(s, n, seed=seed + 1)
    return v[idx], x[idx]


def test_mpmath_spot_values():
    mp.mp.dps = 30
    v, x = _spot_points(48, 104)
    v = np.concatenate([v, [0.0, 0.5, 12.25, 49.99, 30.0]])
    x = np.concatenate([x, [1e-3, 1e3, 12.0, 1e-3, 29.5]])
    ref = np.array([float(mp.log(mp.besselk(mp.mpf(a), mp.mpf(b)))) for a, b in zip(v, x)])
    assert mixed_err(oracle.logk(v, x), ref).max() <= 3e-16


def test_mpmath_spot_derivatives():
    mp.mp.dps = 30
    v, x = _spot_points(12, 105)
    _, dv, dx = oracle.logk(v, x, deriv=True)
    for a, b, d1, d2 in zip(v, x, dv, dx):
        a, b = mp.mpf(a), mp.mpf(b)
        r1 = mp.diff(lambda s: mp.log(mp.besselk(s, b)), a)
        r2 = mp.diff(lambda s: mp.log(mp.besselk(a, s)), b)
        assert abs(d1 - float(r1)) <= 1e-14 * max(1.0, abs(float(r1)))
        assert abs(d2 - float(r2)) <= 1e-14 * max(1.0, abs(float(r2)))


def test_hankel_expansion_with_bound():
    # DLMF 10.40.2 with the remainder bound of DLMF 10.40(ii): for real v, x > 0 and
    # k >= |v| - 1/2 terms, the remainder is at most the first neglected term.
    mp.mp.dps = 40
    for v in [0.0, 0.3, 2.0, 5.5, 9.0]:
        for x in [150.0, 400.0, 1000.0]:
            k = int(math.ceil(abs(v) - 0.5)) + 6
            mu = 4 * mp.mpf(v) ** 2
            terms, a = [], mp.mpf(1)
            for j in range(k + 1):
                if j > 0:
                    a = a * (mu - (2 * j - 1) ** 2) / (j * 8)
                terms.append(a / mp.mpf(x) ** j)
            s = mp.fsum(terms[:-1])
            bound = abs(terms[-1] / s)
            ref = mp.log(mp.sqrt(mp.pi / (2 * x))) - x + mp.log(s)
            got = oracle.logk(v, x)[0]
            assert abs(got - float(ref)) <= float(bound) * 1.01 + 3e-16 * max(1.0, abs(float(ref)))


def debye_logk(v, x):
    """log K_v(x) by the uniform large-order expansion (DLMF 10.41.4, with the
    polynomials u_1..u_3 of DLMF 10.41.10-11), and the size of its last term."""
    v, x = mp.mpf(v), mp.mpf(x)
    z = x / v
    s = mp.sqrt(1 + z * z)
    p = 1 / s
    eta = s + mp.log(z / (1 + s))
    u1 = (3 * p - 5 * p**3) / 24
    u2 = (81 * p**2 - 462 * p**4 + 385 * p**6) / 1152
    u3 = (30375 * p**3 - 369603 * p**5 + 765765 * p**7 - 425425 * p**9) / 414720
    series = 1 - u1 / v + u2 / v**2 - u3 / v**3
    return mp.log(mp.pi / (2 * v)) / 2 - v * eta - mp.log(1 + z * z) / 4 + mp.log(series), abs(u3 / v**3)


def test_large_order_debye():
    # Orders far above the other pins: the truncation interval is then ~1/sqrt(v)
    # wide around a peak at t ~ asinh(v/x).  The expansion's error after u_3 is of
    # the order of u_4 / v^4 (< 1e-15 here); twice the last kept term bounds it.
    mp.mp.dps = 40
    xs = np.array([1e-30, 1e-3, 1.0, 1e2, 1e3, 1e4, 1e5, 1e6])
    for v in [2e3, 1e4, 1e5]:
        lk, dv, dx = oracle.logk(np.full(xs.size, v), xs, deriv=True)
        for i, x in enumerate(xs):
            ref, last = debye_logk(v, x)
            ref_v = mp.diff(lambda q: debye_logk(q, x)[0], v)
            ref_x = mp.diff(lambda q: debye_logk(v, q)[0], x)
            assert abs(lk[i] - float(ref)) <= 2e-15 * max(1.0, abs(float(ref))) + 2 * float(last), (v, x)
            assert mixed_err(dv[i], float(ref_v)) <= 1e-14, (v, x)
            assert mixed_err(dx[i], float(ref_x)) <= 1e-14, (v, x)


def test_large_order_debye_second_derivatives():
    # the oracle's second derivatives against those of the same expansion; the
    # mixed one at x -> 0 (~ -1/x) is the least accurate, 2.9e-11 at v = 1e5
    mp.mp.dps = 40
    xs = np.array([1e-30, 1e-3, 1.0, 1e2, 1e3, 1e4, 1e5, 1e6])
    f = lambda a, b: debye_logk(a, b)[0]  # noqa: E731
    for v in [2e3, 1e4, 1e5]:
        H = oracle.logk_hess(np.full(xs.size, v), xs)
        for i, x in enumerate(xs):
            refs = (mp.diff(f, (v, x), (2, 0)), mp.diff(f, (v, x), (0, 2)), mp.diff(f, (v, x), (1, 1)))
            for k, r in enumerate(refs):
                assert mixed_err(H[i, 3 + k], float(r)) <= 1e-10, (v, x, k)


def test_small_argument_limits():
    # DLMF 10.30.2-3: K_v(x) ~ Gamma(v)/2 (2/x)^v (v > 0), K_0(x) ~ -log(x/2) - gamma.
    x = 1e-3
    for v in [3.0, 5.0, 7.5]:
        lead = math.lgamma(v) - math.log(2) + v * math.log(2 / x)
        rel_corr = x * x / (4 * (v - 1))  # first correction of the finite sum
        assert abs(oracle.logk(v, x)[0] - lead) <= 2 * rel_corr
    x = 1e-6
    k0 = -math.log(x / 2) - np.euler_gamma
    assert abs(math.exp(oracle.logk(0.0, x)[0]) / k0 - 1) <= 1e-10


def test_brute_force_trapezoid():
    # The plain trapezoid with 2^16 bins over the 60-nat interval converges
    # exponentially for this entire, even integrand; it must agree with the adaptive
    # Gauss-Legendre result to double rounding.
    cases = [(0.0, 1e-3), (0.5, 2.0), (3.7, 0.01), (25.0, 24.3), (49.0, 1e-3), (10.0, 900.0), (1.0, 0.9)]
    for v, x in cases:
        _, _, lo, hi = oracle.range_exact(v, x, -60.0)
        brute = oracle.trapezoid_brute(v, x, lo[0], hi[0], 1 << 16)
        lk, dv, dx = oracle.logk(v, x, deriv=True)
        assert mixed_err(brute[0], lk[0]) <= 3e-16
        assert abs(brute[1] - dv[0]) <= 3e-16 * max(1.0, abs(dv[0]))
        assert abs(brute[2] - dx[0]) <= 3e-16 * max(1.0, abs(dx[0]))


def _g(v, x, t):
    z = np.abs(v * t)
    return z + np.log1p(np.exp(-2 * z)) - np.log(2.0) - x * np.cosh(t)


def test_range_exact_invariants():
    v, x, _ = workloads.scale_pairs(2000, seed=106)
    for log_eps in [LOG_EPS64, float(np.log(np.finfo(np.float32).eps))]:
        tp, G, t0, t1 = oracle.range_exact(v, x, log_eps)
        scale = (1.0 + np.abs(G) + abs(log_eps)) * 1e-14  # float64 rounding of g and F
        assert np.all(t0 <= tp) and np.all(tp <= t1)
        assert np.all(np.abs(_g(v, x, tp) - G) <= scale)
        # t_p is a maximum
        for d in (1e-5, 1e-3):
            assert np.all(_g(v, x, tp + d) <= G + scale)
            assert np.all(np.where(tp >= d, _g(v, x, np.maximum(tp - d, 0.0)) <= G + scale, True))
        # peak at 0 exactly when v^2 <= x (Section 2.1)
        assert np.array_equal(tp == 0.0, v * v <= x)
        F = lambda t: _g(v, x, t) - G - log_eps  # noqa: E731
        assert np.all((t0 == 0.0) | (F(t0) <= scale))
        assert np.all(F(t1) <= scale)
        # tight: a step inside each end is inside the set
        assert np.all(F(t1 - 1e-6 * (1 + t1)) >= -scale)
        assert np.all((t0 == 0.0) | (F(t0 + 1e-6 * (1 + t0)) >= -scale))
        # t0 = 0 exactly when g(0) is within the margin (Section 2.3)
        assert np.array_equal(t0 == 0.0, -x - G > log_eps)


def test_method_matches_plain_definition():
    # Algorithms 1-3 + Eq. (int) with integer m reach the integral at n >= 64 bins.
    v, x = workloads.plain_pairs(4096, seed=0)
    ref = oracle.logk(v, x)
    for n, tol in [(64, 5e-13), (128, 1e-15), (256, 1e-15)]:
        lk, _, _, _ = oracle.method_logk(v, x, nbins=n)
        assert mixed_err(lk, ref).max() <= tol, n
    v2, x2, _ = workloads.scale_pairs(8192, seed=107)
    lk, _, _, _ = oracle.method_logk(v2, x2, nbins=128)
    assert mixed_err(lk, oracle.logk(v2, x2)).max() <= 1e-15


def test_method_literal_findrange_fails_small_peak():
    # Reading of Algorithm 1: with m restricted to m >= 0 (as the algorithm box
    # prints it) a peak below t = 1 is bracketed into [1, 2] and n = 64 bins lose
    # accuracy; with m over the integers (Section 2.2's text) they do not.
    v, x = np.array([46.71478737287226]), np.array([979.2244771762067])
    ref = oracle.logk(v, x)
    lit, tp_lit, _, _ = oracle.method_logk(v, x, nbins=64, halve_ok=False)
    fix, tp_fix, _, _ = oracle.method_logk(v, x, nbins=64, halve_ok=True)
    assert mixed_err(lit, ref)[0] > 1e-9
    assert mixed_err(fix, ref)[0] <= 1e-14
    assert tp_lit[0] >= 1.0 and tp_fix[0] < 0.2


def test_domain_conventions():
    v = np.array([np.nan, 1.0, 1.0, 1.0, 1.0, np.inf, -np.inf])
    x = np.array([1.0, np.nan, -1.0, 0.0, np.inf, 2.0, 2.0])
    lk, dv, dx = oracle.logk(v, x, deriv=True)
    assert np.isnan(lk[0]) and np.isnan(lk[1]) and np.isnan(lk[2])
    assert lk[3] == np.inf and lk[4] == -np.inf
    assert lk[5] == np.inf and lk[6] == np.inf
    assert np.all(np.isnan(dv)) and np.all(np.isnan(dx))


@pytest.mark.parametrize("bad", ["n", "eps"])
def test_argument_errors(bad):
    with pytest.raises(ValueError):
        if bad == "eps":
            oracle.range_exact([1.0], [1.0], 0.5)
        else:
            oracle.method_logk([1.0], [1.0], nbins=0)
