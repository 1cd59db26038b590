"""Pins of the oracle's second derivatives of log K (oracle_logk_hess_batch).

* the modified Bessel equation x^2 K'' + x K' - (x^2 + v^2) K = 0 (DLMF 10.25.1)
  ties d2/dx2 log K to d/dx log K, which other pins fix;
* the closed form K_{1/2}(x) = sqrt(pi / (2x)) e^{-x} (DLMF 10.39.2);
* Richardson-extrapolated central differences of the oracle's own first
  derivatives, in v and in x (the mixed derivative both ways);
* log K as a cumulant generating function: with the even extension,
  K_v(x) = 1/2 int_R e^{v t} e^{-x cosh t} dt, so d2/dv2 log K is a variance of
  t and d2/dx2 log K one of cosh t: both positive;
* evenness in v of d2/dv2 and d2/dx2, oddness of d2/dvdx, and d2/dvdx = 0 at v = 0.
"""

import numpy as np
import pytest

import oracle

V = np.array([0.0, 0.5, 1.3, 2.5, 10.0, 30.0, 49.0])
X = np.array([1e-3, 0.05, 0.7, 3.0, 30.0, 400.0, 1e3])
VG, XG = (a.ravel() for a in np.meshgrid(V, X, indexing="ij"))


@pytest.fixture(scope="module")
def H():
    return oracle.logk_hess(VG, XG)


def test_first_derivatives_unchanged(H):
    lk, dv, dx = oracle.logk(VG, XG, deriv=True)
    assert np.array_equal(H[:, 0], lk)
    assert np.array_equal(H[:, 1], dv)
    assert np.array_equal(H[:, 2], dx)


def test_bessel_equation(H):
    dx, d2x = H[:, 2], H[:, 4]
    # K''/K = d2x + dx^2;  x^2 K''/K + x K'/K - (x^2 + v^2) = 0
    terms = np.stack([XG ** 2 * d2x, XG ** 2 * dx ** 2, XG * dx, XG ** 2, VG ** 2])
    resid = XG ** 2 * (d2x + dx ** 2) + XG * dx - (XG ** 2 + VG ** 2)
    scale = np.abs(terms).max(axis=0)
    assert np.max(np.abs(resid) / scale) <= 1e-14


def test_half_order_closed_form():
    x = np.geomspace(1e-3, 1e3, 25)
    H = oracle.logk_hess(np.full_like(x, 0.5), x)
    # log K = 1/2 log(pi/2) - 1/2 log x - x:  d/dx = -1/(2x) - 1,  d2/dx2 = 1/(2 x^2)
    np.testing.assert_allclose(H[:, 2], -0.5 / x - 1.0, rtol=1e-15, atol=0)
    ref = 0.5 / x ** 2
    # mixed error: at large x the variance of cosh t is ~1/(2x^2) against
    # E[cosh^2 t] ~ 1, so its relative accuracy is that of 1, not of the variance
    assert np.max(np.abs(H[:, 4] - ref) / np.maximum(1.0, ref)) <= 1e-14


def _richardson(f, z, h):
    d1 = (f(z + h) - f(z - h)) / (2 * h)
    d2 = (f(z + h / 2) - f(z - h / 2)) / h
    return (4 * d2 - d1) / 3


def test_second_derivative_in_v_by_differences(H):
    sel = VG >= 0.5  # keep v - h on the same side of 0
    v, x = VG[sel], XG[sel]
    h = 2e-3

    def dv_at(vv):
        return oracle.logk(vv, x, deriv=True)[1]

    fd = _richardson(dv_at, v, h)
    err = np.abs(fd - H[sel, 3]) / np.maximum(1.0, np.abs(H[sel, 3]))
    assert err.max() <= 1e-10


def test_mixed_derivative_both_ways(H):
    sel = VG >= 0.5
    v, x = VG[sel], XG[sel]
    hx = 1e-3 * x
    fd_x = _richardson(lambda xx: oracle.logk(v, xx, deriv=True)[1], x, hx)
    fd_v = _richardson(lambda vv: oracle.logk(vv, x, deriv=True)[2], v, 2e-3)
    ref = H[sel, 5]
    scale = np.maximum(1.0, np.abs(ref))
    assert (np.abs(fd_x - ref) / scale).max() <= 1e-10
    assert (np.abs(fd_v - ref) / scale).max() <= 1e-10


def test_second_derivative_in_x_by_differences(H):
    x = XG
    hx = 1e-3 * x
    fd = _richardson(lambda xx: oracle.logk(VG, xx, deriv=True)[2], x, hx)
    err = np.abs(fd - H[:, 4]) / np.maximum(1.0, np.abs(H[:, 4]))
    assert err.max() <= 1e-10


def test_variances_are_positive(H):
    assert np.all(H[:, 3] > 0.0)
    assert np.all(H[:, 4] > 0.0)


def test_parity_in_v():
    v = np.array([0.7, 2.5, 12.0])
    x = np.array([0.3, 3.0, 50.0])
    P = oracle.logk_hess(v, x)
    N = oracle.logk_hess(-v, x)
    assert np.array_equal(P[:, [0, 2, 3, 4]], N[:, [0, 2, 3, 4]])
    assert np.array_equal(P[:, [1, 5]], -N[:, [1, 5]])
    Z = oracle.logk_hess(np.zeros(3), x)
    assert np.all(Z[:, 1] == 0.0) and np.all(Z[:, 5] == 0.0)
    assert np.all(Z[:, 3] > 0.0)


def test_domain_conventions():
    nan, inf = float("nan"), float("inf")
    v = np.array([nan, 1.0, 1.0, 1.0, 1.0, inf])
    x = np.array([1.0, nan, -1.0, 0.0, inf, 2.0])
    H = oracle.logk_hess(v, x)
    assert np.isnan(H[:3]).all()
    assert H[3, 0] == inf and H[4, 0] == -inf and H[5, 0] == inf
    assert np.isnan(H[3:, 1:]).all()
