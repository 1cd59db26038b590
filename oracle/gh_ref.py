"""Reference per-set sums of the generalised-hyperbolic-shaped batch (test only).

For parameter sets i and shared samples y_j:
    v_ij = lambda_i - 1/2,   r_ij = sqrt(delta_i^2 + (y_j - mu_i)^2),   x_ij = alpha_i r_ij,
    S_i  = sum_j log K_{v_ij}(x_ij)
and the gradient of S_i (times an optional upstream gradient g_i) by the chain
rule through d/dv log K and d/dx log K of the oracle:
    dS/dlambda = sum_j dv_ij,          dS/dalpha = sum_j dx_ij r_ij,
    dS/ddelta  = sum_j dx_ij alpha delta / r_ij,
    dS/dmu     = sum_j dx_ij alpha (mu - y_j) / r_ij.
Sums in long double via math.fsum-like compensated numpy (np.sum over float64
pairs is enough at these sizes; fsum is used for the sums themselves).
"""

from __future__ import annotations

import math

import numpy as np

import oracle


def gh_sums(lam, alpha, delta, mu, y, gsum=None, nthreads=None, with_scales=False):
    """(S, dS/dlambda, dS/dalpha, dS/ddelta, dS/dmu) per set; with_scales also
    returns, per output, sum_j max(1, |term_j|) (times |g_i| for the gradients):
    the natural scale of a sum's rounding, for tolerances."""
    lam, alpha, delta, mu = (np.asarray(a, dtype=np.float64) for a in (lam, alpha, delta, mu))
    y = np.asarray(y, dtype=np.float64)
    S = lam.size
    v = np.repeat(lam - 0.5, y.size)
    dy = y[None, :] - mu[:, None]
    r = np.sqrt(delta[:, None] ** 2 + dy * dy)
    x = (alpha[:, None] * r).ravel()
    lk, dv, dx = oracle.logk(v, x, deriv=True, nthreads=nthreads)
    lk, dv, dx = (a.reshape(S, y.size) for a in (lk, dv, dx))
    out = np.array([math.fsum(row) for row in lk])
    g_lam = np.array([math.fsum(row) for row in dv])
    g_alpha = np.array([math.fsum(row) for row in dx * r])
    g_delta = np.array([math.fsum(row) for row in dx * alpha[:, None] * delta[:, None] / r])
    g_mu = np.array([math.fsum(row) for row in dx * alpha[:, None] * (-dy) / r])
    terms = (lk, dv, dx * r, dx * alpha[:, None] * delta[:, None] / r, dx * alpha[:, None] * (-dy) / r)
    sc = [np.maximum(1.0, np.abs(t)).sum(axis=1) for t in terms]
    if gsum is not None:
        g = np.asarray(gsum, dtype=np.float64)
        g_lam, g_alpha, g_delta, g_mu = g * g_lam, g * g_alpha, g * g_delta, g * g_mu
        sc = sc[:1] + [np.abs(g) * c for c in sc[1:]]
    if with_scales:
        return (out, g_lam, g_alpha, g_delta, g_mu), sc
    return out, g_lam, g_alpha, g_delta, g_mu
