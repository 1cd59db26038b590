"""GPU per-set sums (bessel_gh_logk_sum) against the FP64 reference (oracle/gh_ref.py).

Tolerance per set: the FP32 elementwise bar (1e-5 mixed error) summed over the
set's samples, i.e. 1e-5 * sum_j max(1, |term_j|) for the sum and for each
gradient component.
"""

import numpy as np
import pytest
import torch

import oracle
import workloads
from oracle import gh_ref

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def bk():
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a GPU")
    import paper_2108_11560_amd as mod
    mod.load()
    return mod


def dev32(a):
    return torch.tensor(np.asarray(a), dtype=torch.float32, device="cuda")


def host(t):
    return t.double().cpu().numpy()


def f32(a):
    return np.asarray(a, dtype=np.float32).astype(np.float64)


def scales(lam, alpha, delta, mu, y):
    """sum_j max(1, |term_j|) per set for the five outputs (tolerance scales)."""
    v = np.repeat(lam - 0.5, y.size)
    dy = y[None, :] - mu[:, None]
    r = np.sqrt(delta[:, None] ** 2 + dy * dy)
    lk, dv, dx = oracle.logk(v, (alpha[:, None] * r).ravel(), deriv=True)
    S = lam.size
    lk, dv, dx = (a.reshape(S, y.size) for a in (lk, dv, dx))
    terms = [lk, dv, dx * r, dx * alpha[:, None] * delta[:, None] / r, dx * alpha[:, None] * dy / r]
    return [np.maximum(1.0, np.abs(t)).sum(axis=1) for t in terms]


def check_against_reference(got, lam, alpha, delta, mu, y, gs):
    ref = gh_ref.gh_sums(lam, alpha, delta, mu, y, gs)
    sc = scales(lam, alpha, delta, mu, y)
    for k in range(5):
        g = np.abs(gs) if (gs is not None and k > 0) else 1.0
        assert np.all(np.abs(host(got[k]) - ref[k]) <= 1e-5 * sc[k] * g), k


def test_all_sets_256_samples(bk):
    lam, alpha, delta, mu, y, gs = workloads.gh_batch(1024, 65536, seed=5, grad_seed=15)
    lam, alpha, delta, mu, y, gs = (f32(a) for a in (lam, alpha, delta, mu, y, gs))
    y = y[:256]
    got = bk.gh_logk_sum(dev32(lam), dev32(alpha), dev32(delta), dev32(mu), dev32(y), grad_sum=dev32(gs))
    check_against_reference(got, lam, alpha, delta, mu, y, gs)


def test_full_sets_at_scale(bk):
    # the full 1024 x 65536 batch on the GPU; the oracle checks four whole sets
    lam, alpha, delta, mu, y, gs = workloads.gh_batch(1024, 65536, seed=5, grad_seed=15)
    lam, alpha, delta, mu, y, gs = (f32(a) for a in (lam, alpha, delta, mu, y, gs))
    got = bk.gh_logk_sum(dev32(lam), dev32(alpha), dev32(delta), dev32(mu), dev32(y), grad_sum=dev32(gs))
    assert all(bool(torch.isfinite(g).all()) for g in got)
    pick = np.array([0, 311, 702, 1023])
    sub = [g[torch.tensor(pick, device="cuda")] for g in got]
    check_against_reference(sub, lam[pick], alpha[pick], delta[pick], mu[pick], y, gs[pick])


def test_matches_elementwise_path(bk):
    lam, alpha, delta, mu, y, _ = workloads.gh_batch(8, 3000, seed=33)
    lam, alpha, delta, mu, y = (f32(a) for a in (lam, alpha, delta, mu, y))
    S, gl, ga, gd, gm = bk.gh_logk_sum(dev32(lam), dev32(alpha), dev32(delta), dev32(mu), dev32(y))
    v = np.repeat(lam - 0.5, y.size)
    dy = y[None, :] - mu[:, None]
    r = np.sqrt(delta[:, None] ** 2 + dy * dy)
    x = (alpha[:, None] * r).astype(np.float32)
    lk, dv, dx = bk.logk_dv_dx(dev32(v), dev32(x.ravel()))
    lk = host(lk).reshape(8, -1)
    # elementwise outputs are rounded to FP32 (relative 6e-8) and x was rounded too
    assert np.all(np.abs(host(S) - lk.sum(axis=1)) <= 1e-6 * np.abs(lk).sum(axis=1) + 1e-6 * y.size)


def test_upstream_gradient_scales(bk):
    lam, alpha, delta, mu, y, gs = workloads.gh_batch(64, 2048, seed=34, grad_seed=35)
    args = [dev32(a) for a in (lam, alpha, delta, mu, y)]
    plain = bk.gh_logk_sum(*args)
    scaled = bk.gh_logk_sum(*args, grad_sum=dev32(gs))
    assert torch.equal(plain[0], scaled[0])
    for k in range(1, 5):
        assert np.allclose(host(scaled[k]), host(plain[k]) * f32(gs), rtol=2e-7, atol=0)


def test_deterministic(bk):
    lam, alpha, delta, mu, y, gs = workloads.gh_batch(256, 8192, seed=36)
    args = [dev32(a) for a in (lam, alpha, delta, mu, y)]
    a = bk.gh_logk_sum(*args, grad_sum=dev32(gs))
    b = bk.gh_logk_sum(*args, grad_sum=dev32(gs))
    assert all(torch.equal(p, q) for p, q in zip(a, b))


def test_ragged_and_empty(bk):
    lam, alpha, delta, mu, y, _ = workloads.gh_batch(3, 1000, seed=37)
    lam, alpha, delta, mu, y = (f32(a) for a in (lam, alpha, delta, mu, y))
    for ns in (1, 255, 257, 1000):
        got = bk.gh_logk_sum(dev32(lam), dev32(alpha), dev32(delta), dev32(mu), dev32(y[:ns]))
        check_against_reference(got, lam, alpha, delta, mu, y[:ns], None)
    empty = bk.gh_logk_sum(dev32(lam), dev32(alpha), dev32(delta), dev32(mu), dev32(np.zeros(0)))
    assert np.all(host(empty[0]) == 0.0)


# ---- the bracket from the network's table (range="mlp_table") --------------


@pytest.fixture(scope="module")
def net(bk):
    """A predictor trained and calibrated as the benchmark's (2^20 scale pairs,
    20 000 Adam steps, margins on 2^16 held-out pairs)."""
    from paper_2108_11560_amd import mlp as M
    m = M.RangeMLP(M.glorot_params(0))
    v, x, _ = workloads.scale_pairs(1 << 20, seed=4)
    m.train(dev32(v), dev32(x), steps=20000, batch=8192, lr=3e-3, lr_final=3e-5, seed=1)
    vc, xc, _ = workloads.scale_pairs(1 << 16, seed=8)
    M.calibrate_margins(m, dev32(vc), dev32(xc), range="mlp_table")
    yield m
    m.close()


def test_table_range_all_sets_256_samples(bk, net):
    lam, alpha, delta, mu, y, gs = workloads.gh_batch(1024, 65536, seed=5, grad_seed=15)
    lam, alpha, delta, mu, y, gs = (f32(a) for a in (lam, alpha, delta, mu, y, gs))
    y = y[:256]
    got = bk.gh_logk_sum(dev32(lam), dev32(alpha), dev32(delta), dev32(mu), dev32(y), grad_sum=dev32(gs),
                         range="mlp_table", mlp=net)
    check_against_reference(got, lam, alpha, delta, mu, y, gs)


def test_table_range_full_sets_at_scale(bk, net):
    lam, alpha, delta, mu, y, gs = workloads.gh_batch(1024, 65536, seed=5, grad_seed=15)
    lam, alpha, delta, mu, y, gs = (f32(a) for a in (lam, alpha, delta, mu, y, gs))
    args = [dev32(a) for a in (lam, alpha, delta, mu, y)]
    got = bk.gh_logk_sum(*args, grad_sum=dev32(gs), range="mlp_table", mlp=net)
    newton = bk.gh_logk_sum(*args, grad_sum=dev32(gs))
    assert all(bool(torch.isfinite(g).all()) for g in got)
    pick = np.array([0, 311, 702, 1023])
    sub = [g[torch.tensor(pick, device="cuda")] for g in got]
    check_against_reference(sub, lam[pick], alpha[pick], delta[pick], mu[pick], y, gs[pick])
    # against the Newton bracket on every set: both within the FP32 bar of
    # the exact sums, so within twice that of each other
    sc = scales(lam[pick], alpha[pick], delta[pick], mu[pick], y)
    for k in range(5):
        d = np.abs(host(got[k]) - host(newton[k]))[pick]
        g = np.abs(gs[pick]) if k > 0 else 1.0
        assert np.all(d <= 2e-5 * sc[k] * g), k


def test_table_range_forced_fallback_is_the_newton_sum(bk):
    # zero weights with a t1 margin of -30: every learned bracket fails its
    # check and takes the Newton bracket in its lane, so the sums are those of
    # the Newton call bit for bit
    from paper_2108_11560_amd import mlp as M
    p = np.zeros(M.NPARAMS, dtype=np.float32)
    p[M.O_META:M.O_META + 6] = [1.0, 3.0, 0.0, 4.0, -30.0, 0.0]
    m = M.RangeMLP(p)
    try:
        lam, alpha, delta, mu, y, gs = workloads.gh_batch(64, 3000, seed=38, grad_seed=39)
        args = [dev32(a) for a in (lam, alpha, delta, mu, y)]
        a = bk.gh_logk_sum(*args, grad_sum=dev32(gs), range="mlp_table", mlp=m)
        b = bk.gh_logk_sum(*args, grad_sum=dev32(gs))
        assert all(torch.equal(p_, q_) for p_, q_ in zip(a, b))
    finally:
        m.close()


def test_table_range_no_alloc_matches(bk, net):
    lam, alpha, delta, mu, y, gs = workloads.gh_batch(128, 4096, seed=40, grad_seed=41)
    args = [dev32(a) for a in (lam, alpha, delta, mu, y)]
    a = bk.gh_logk_sum(*args, grad_sum=dev32(gs), range="mlp_table", mlp=net)
    b = bk.gh_logk_sum(*args, grad_sum=dev32(gs), range="mlp_table", mlp=net, no_alloc=True)
    assert all(torch.equal(p_, q_) for p_, q_ in zip(a, b))


def test_learned_range_modes_rejected_or_required(bk, net):
    lam, alpha, delta, mu, y, _ = workloads.gh_batch(4, 100, seed=42)
    args = [dev32(a) for a in (lam, alpha, delta, mu, y)]
    with pytest.raises(RuntimeError, match="UNSUPPORTED"):
        bk.gh_logk_sum(*args, range="mlp", mlp=net)
    with pytest.raises(RuntimeError, match="RANGE_MODE"):
        bk.gh_logk_sum(*args, range="mlp_table")
