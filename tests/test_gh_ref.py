"""Pins of the per-set reference (oracle/gh_ref.py): its chain rule against
central differences of its own sums in each parameter, and the v = -v symmetry."""

import numpy as np

import workloads
from oracle import gh_ref


def test_chain_rule_matches_central_differences():
    lam, alpha, delta, mu, y, g = workloads.gh_batch(nsets=5, nsamp=7, seed=31)
    S, gl, ga, gd, gm = gh_sums = gh_ref.gh_sums(lam, alpha, delta, mu, y, g)
    h = 1e-6
    for name, base, grad in [("lam", lam, gl), ("alpha", alpha, ga), ("delta", delta, gd), ("mu", mu, gm)]:
        for i in range(lam.size):
            args = {"lam": lam, "alpha": alpha, "delta": delta, "mu": mu}
            up = {k: a.copy() for k, a in args.items()}
            dn = {k: a.copy() for k, a in args.items()}
            up[name][i] += h
            dn[name][i] -= h
            fd = (gh_ref.gh_sums(y=y, **up)[0][i] - gh_ref.gh_sums(y=y, **dn)[0][i]) / (2 * h) * g[i]
            assert abs(fd - grad[i]) <= 1e-6 * max(1.0, abs(grad[i])), (name, i)


def test_order_symmetry():
    # lambda -> 1 - lambda maps v -> -v: the sums agree and dS/dlambda flips sign
    lam, alpha, delta, mu, y, _ = workloads.gh_batch(nsets=4, nsamp=9, seed=32)
    a = gh_ref.gh_sums(lam, alpha, delta, mu, y)
    b = gh_ref.gh_sums(1.0 - lam, alpha, delta, mu, y)
    assert np.allclose(a[0], b[0], rtol=1e-15, atol=0)
    assert np.allclose(a[1], -b[1], rtol=1e-13, atol=1e-15)


def test_scales_bound_the_sums():
    # sum_j max(1, |term_j|) >= |sum_j term_j| (with |g| on the gradients), and
    # asking for the scales leaves the sums as they are
    lam, alpha, delta, mu, y, g = workloads.gh_batch(nsets=6, nsamp=11, seed=33)
    plain = gh_ref.gh_sums(lam, alpha, delta, mu, y, g)
    sums, sc = gh_ref.gh_sums(lam, alpha, delta, mu, y, g, with_scales=True)
    for k in range(5):
        assert np.array_equal(plain[k], sums[k])
        assert np.all(sc[k] >= np.abs(sums[k]) * (1 - 1e-12))
    assert np.all(sc[0] >= y.size)
