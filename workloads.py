"""Seeded synthetic inputs for log K_v(x) workloads.

This module only draws random numbers; it holds none of the method's arithmetic.
Both the GPU library's tests/benchmark and the CPU oracle's tests take their
inputs from here.  Every generator uses ``numpy.random.default_rng(seed)``
(PCG64), draws in float64, and draws the order v, then x, then band choices.
FP32 inputs are the float64 draws rounded to nearest.

Shapes and distributions follow the paper's evaluation domain (Section 3:
v in [0, 99], x in [10^-1, 10^2.1]; batch sweep with v = 10^{2r} - 1,
x = 10^{3r - 1}) widened to the benchmark workloads below.
"""

from __future__ import annotations

import numpy as np

# ---------------------------------------------------------------------------
# Named workloads
# ---------------------------------------------------------------------------

PLAIN_4096 = dict(name="plain-fp64-4096", n=4096, seed=0)
SCALE_2P24 = dict(name="scale-2^24", n=1 << 24, seed=1)
DIFF_2P22 = dict(name="diff-2^22", n=1 << 22, seed=3, grad_seed=13)
MLP_TRAIN_2P20 = dict(name="mlp-train-2^20", n=1 << 20, seed=4)
GH_1024x65536 = dict(name="gh-1024x65536", nsets=1024, nsamp=65536, seed=5, grad_seed=15)


def plain_pairs(n: int = 4096, seed: int = 0):
    """v ~ U[0, 10], x ~ 10^U[-2, 2] (float64)."""
    rng = np.random.default_rng(seed)
    v = rng.uniform(0.0, 10.0, n)
    x = 10.0 ** rng.uniform(-2.0, 2.0, n)
    return v, x


def scale_pairs(n: int = 1 << 24, seed: int = 1):
    """Wide domain with hard bands, randomly permuted (float64).

    75 %:    v ~ U[0, 50], x ~ 10^U[-3, 3]
    12.5 %:  band A (|v - x| < 1): v ~ U[0, 50], x ~ U[max(1e-3, v - 1), v + 1]
    12.5 %:  band B (v > 20, x < 0.1): v ~ U[20, 50], x ~ 10^U[-3, -1]
    """
    rng = np.random.default_rng(seed)
    n_a = n // 8
    n_b = n // 8
    n_m = n - n_a - n_b
    v_m = rng.uniform(0.0, 50.0, n_m)
    x_m = 10.0 ** rng.uniform(-3.0, 3.0, n_m)
    v_a = rng.uniform(0.0, 50.0, n_a)
    lo = np.maximum(1e-3, v_a - 1.0)
    x_a = rng.uniform(lo, v_a + 1.0)
    v_b = rng.uniform(20.0, 50.0, n_b)
    x_b = 10.0 ** rng.uniform(-3.0, -1.0, n_b)
    v = np.concatenate([v_m, v_a, v_b])
    x = np.concatenate([x_m, x_a, x_b])
    stratum = np.concatenate([np.zeros(n_m, np.int8), np.ones(n_a, np.int8), np.full(n_b, 2, np.int8)])
    perm = rng.permutation(n)
    return v[perm], x[perm], stratum[perm]


def stratified_subset(stratum: np.ndarray, k: int, seed: int = 11):
    """Indices of a k-element subset with equal counts from every stratum."""
    rng = np.random.default_rng(seed)
    labels = np.unique(stratum)
    per = k // len(labels)
    out = []
    for s in labels:
        idx = np.flatnonzero(stratum == s)
        out.append(rng.choice(idx, size=min(per, idx.size), replace=False))
    return np.sort(np.concatenate(out))


def upstream_grad(n: int, seed: int = 13):
    """Upstream gradients ~ N(0, 1) (float64)."""
    return np.random.default_rng(seed).standard_normal(n)


def gh_batch(nsets: int = 1024, nsamp: int = 65536, seed: int = 5, grad_seed: int = 15):
    """Generalised-hyperbolic-likelihood-shaped batch (float64).

    lambda ~ U[-3, 3], alpha ~ exp(U[ln 0.5, ln 20]), delta ~ exp(U[ln 0.1, ln 5]),
    mu ~ N(0, 1) per set; y ~ N(0, variance 4) shared by all sets; upstream
    gradient on each per-set sum ~ N(0, 1).
    """
    rng = np.random.default_rng(seed)
    lam = rng.uniform(-3.0, 3.0, nsets)
    alpha = np.exp(rng.uniform(np.log(0.5), np.log(20.0), nsets))
    delta = np.exp(rng.uniform(np.log(0.1), np.log(5.0), nsets))
    mu = rng.standard_normal(nsets)
    y = 2.0 * rng.standard_normal(nsamp)
    gsum = np.random.default_rng(grad_seed).standard_normal(nsets)
    return lam, alpha, delta, mu, y, gsum


def paper_sweep(n: int, seed: int = 21):
    """The paper's batch-size sweep: v = 10^{2r} - 1, x = 10^{3r'-1}, r, r' ~ U[0, 1]."""
    rng = np.random.default_rng(seed)
    v = 10.0 ** (2.0 * rng.uniform(0.0, 1.0, n)) - 1.0
    x = 10.0 ** (3.0 * rng.uniform(0.0, 1.0, n) - 1.0)
    return v, x


def accuracy_grid():
    """The paper's accuracy grid (Section 3.1): v = 10^{i/40} - 1 (i = 0..80),
    x = 10^{j/40 - 1} (j = 0..124), as flattened (v, x) with v varying slowest."""
    vv = 10.0 ** (np.arange(81) / 40.0) - 1.0
    xx = 10.0 ** (np.arange(125) / 40.0 - 1.0)
    V, X = np.meshgrid(vv, xx, indexing="ij")
    return V.ravel(), X.ravel()


def domain_pairs(n: int, seed: int = 31):
    """Pairs across the validated FP64 domain: half with v ~ U[0, 1e3], half
    with v ~ LogU[1e-8, 1] (orders near 0), x ~ LogU[1e-6, 1e5] throughout;
    the two halves interleaved."""
    rng = np.random.default_rng(seed)
    big = rng.uniform(0.0, 1e3, n)
    small = 10.0 ** rng.uniform(-8.0, 0.0, n)
    v = np.where(np.arange(n) % 2 == 0, big, small)
    x = 10.0 ** rng.uniform(-6.0, 5.0, n)
    return v, x


def to_f32(a: np.ndarray) -> np.ndarray:
    """Round float64 draws to the nearest float32."""
    return np.asarray(a, dtype=np.float64).astype(np.float32)
