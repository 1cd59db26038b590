"""GPU parity of the small-batch kernels (16 lanes per element; batches up to
the split threshold) against the oracle, and their agreement with the
one-lane-per-element kernels on the same inputs.

Tolerances: the path's bars (mixed error, FP64 1e-12, FP32 1e-5) against the
oracle; between the two layouts 1e-13 (FP64) and 2e-7 (FP32, a few FP32
roundings of the output).  The layouts add the same terms in a different
order and start their recurrences (e^{t} products, cosh t, 1 - e^{-2vt}) at
different nodes, so the node arguments differ by a few ulp of x cosh t.
"""

import numpy as np
import pytest
import torch

import oracle
import workloads

pytestmark = pytest.mark.gpu

TOL = {torch.float64: 1e-12, torch.float32: 1e-5}
AGREE = {torch.float64: 1e-13, torch.float32: 2e-7}


@pytest.fixture(scope="module")
def bk():
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a GPU")
    import paper_2108_11560_amd as mod
    mod.load()
    return mod


def mixed(a, b):
    return np.abs(np.asarray(a, np.float64) - b) / np.maximum(1.0, np.abs(b))


def dev(a, dt):
    return torch.tensor(np.asarray(a), dtype=dt, device="cuda")


def host(t):
    return t.double().cpu().numpy()


class threshold:
    def __init__(self, bk, n):
        self.bk, self.n = bk, n

    def __enter__(self):
        self.prev = self.bk.set_split_threshold(self.n)

    def __exit__(self, *exc):
        self.bk.set_split_threshold(self.prev)


@pytest.mark.parametrize("dt", [torch.float64, torch.float32])
@pytest.mark.parametrize("n", [1, 15, 17, 1000, 4097])
def test_small_batches_against_oracle(bk, dt, n):
    v, x, _ = workloads.scale_pairs(n, seed=500 + n)
    vt, xt = dev(v, dt), dev(x, dt)
    with threshold(bk, 1 << 20):
        lk, dv, dx = bk.logk_dv_dx(vt, xt)
        lk0 = bk.logk(vt, xt)
    ref, rdv, rdx = oracle.logk(host(vt), host(xt), deriv=True)
    assert mixed(host(lk), ref).max() <= TOL[dt]
    assert mixed(host(dv), rdv).max() <= TOL[dt]
    assert mixed(host(dx), rdx).max() <= TOL[dt]
    assert torch.equal(lk, lk0)  # forward and derivative kernels: same S0


@pytest.mark.parametrize("nbins", [2, 7, 16, 64, 100, 256, 1000])
def test_bin_counts_including_fewer_than_lanes(bk, nbins):
    v, x = workloads.plain_pairs(500, seed=21)
    vt, xt = dev(v, torch.float64), dev(x, torch.float64)
    with threshold(bk, 1 << 20):
        split = bk.logk_dv_dx(vt, xt, nbins=nbins)
    with threshold(bk, 0):
        one = bk.logk_dv_dx(vt, xt, nbins=nbins)
    for a, b in zip(split, one):
        a, b = host(a), host(b)
        assert mixed(a, b).max() <= (AGREE[torch.float64] if nbins >= 64 else 1e-12)
    if nbins >= 64:
        assert mixed(host(split[0]), oracle.logk(v, x)).max() <= 1e-12


@pytest.mark.parametrize("dt", [torch.float64, torch.float32])
def test_layouts_agree_on_scale_pairs(bk, dt):
    v, x, _ = workloads.scale_pairs(1 << 16, seed=33)
    vt, xt = dev(v, dt), dev(x, dt)
    go = dev(workloads.upstream_grad(1 << 16, seed=34), dt)
    with threshold(bk, 1 << 20):
        split = bk.logk_dv_dx(vt, xt, grad_out=go)
    with threshold(bk, 0):
        one = bk.logk_dv_dx(vt, xt, grad_out=go)
    for a, b in zip(split, one):
        assert mixed(host(a), host(b)).max() <= AGREE[dt]


def test_domain_conventions_split(bk):
    nan, inf = float("nan"), float("inf")
    v = dev([nan, 1.0, 1.0, 1.0, 1.0, inf, 2.5, -2.5, 0.0], torch.float64)
    x = dev([1.0, nan, -1.0, 0.0, inf, 2.0, 3.0, 3.0, 3.0], torch.float64)
    with threshold(bk, 1 << 20):
        lk, dv, dx = (host(t) for t in bk.logk_dv_dx(v, x))
    assert np.isnan(lk[:3]).all()
    assert lk[3] == np.inf and lk[4] == -np.inf and lk[5] == np.inf
    assert lk[6] == lk[7] and dv[6] == -dv[7] and dv[8] == 0.0


def test_threshold_policy(bk):
    prev = bk.set_split_threshold(123)
    assert bk.set_split_threshold(prev) == 123
    with pytest.raises(bk.BesselError):
        bk.set_split_threshold(-1)


# ---- second derivatives on the 16-lane layout ------------------------------

HESS_AGREE = {torch.float64: 1e-12, torch.float32: 2e-6}


@pytest.mark.parametrize("dt", [torch.float64, torch.float32])
@pytest.mark.parametrize("n", [1, 15, 17, 1000, 4097])
def test_hess_small_batches_against_oracle(bk, dt, n):
    v, x, _ = workloads.scale_pairs(n, seed=520 + n)
    vt, xt = dev(v, dt), dev(x, dt)
    with threshold(bk, 1 << 20):
        got = np.stack([host(o) for o in bk.logk_hess(vt, xt)], axis=1)
    ref = oracle.logk_hess(host(vt), host(xt))
    err = mixed(got, ref)
    assert err.max() <= TOL[dt], err.max(axis=0)
    # the one-lane layout on the same inputs: the same sums in another order
    with threshold(bk, 0):
        one = np.stack([host(o) for o in bk.logk_hess(vt, xt)], axis=1)
    assert mixed(got, one).max() <= HESS_AGREE[dt]


def test_hess_split_validated_domain(bk):
    # the centred FP64 moments on the split layout across the validated
    # domain (v to 1e3, x in [1e-6, 1e5]), against the oracle at the FP64 bar
    v, x = workloads.domain_pairs(400, seed=62)
    vt, xt = dev(v, torch.float64), dev(x, torch.float64)
    with threshold(bk, 1 << 20):
        got = np.stack([host(o) for o in bk.logk_hess(vt, xt)], axis=1)
    ref = oracle.logk_hess(v, x)
    err = mixed(got, ref)
    print("split layout, validated domain: max mixed error per output", err.max(axis=0))
    assert err.max() <= 1e-12


def test_hess_split_conventions(bk):
    nan, inf = float("nan"), float("inf")
    v = dev([nan, 1.0, 1.0, 1.0, 1.0, inf, -2.5, 0.0], torch.float64)
    x = dev([1.0, nan, -1.0, 0.0, inf, 2.0, 3.0, 3.0], torch.float64)
    with threshold(bk, 1 << 20):
        out = [host(o) for o in bk.logk_hess(v, x)]
        pos = [host(o) for o in bk.logk_hess(-v[6:7], x[6:7])]
    assert np.isnan(out[0][:3]).all()
    assert out[0][3] == inf and out[0][4] == -inf and out[0][5] == inf
    for o in out[1:]:
        assert np.isnan(o[:6]).all()
    # odd in v: d/dv and d2/dvdx flip sign, the rest do not; v = 0 gives 0
    assert pos[1][0] == -out[1][6] and pos[5][0] == -out[5][6]
    assert pos[3][0] == out[3][6] and pos[4][0] == out[4][6]
    assert out[1][7] == 0.0 and out[5][7] == 0.0


# ---- learned range modes below the threshold -------------------------------


@pytest.mark.parametrize("mode", ["mlp", "mlp_table"])
@pytest.mark.parametrize("n", [1, 15, 17, 1000, 4097])
def test_learned_small_batches_take_the_split_newton_path(bk, mode, n):
    """At most the split threshold, a learned-range call runs the Newton
    bracket on 16 lanes per element (one launch), so its results are those of
    the plain FP32 call on the same layout, bit for bit, and the handle
    reports no fallback."""
    from paper_2108_11560_amd import mlp as M
    v, x, _ = workloads.scale_pairs(n, seed=540 + n)
    vt, xt = dev(v, torch.float32), dev(x, torch.float32)
    go = dev(workloads.upstream_grad(n, seed=541 + n), torch.float32)
    # zero weights and a t1 margin of -30: every learned bracket fails its
    # check, so a call on the fused kernel would count n fallbacks
    p = np.zeros(M.NPARAMS, dtype=np.float32)
    p[M.O_META:M.O_META + 6] = [1.0, 3.0, 0.0, 4.0, -30.0, 0.0]
    mlp = M.RangeMLP(p)
    try:
        with threshold(bk, 0):
            bk.logk(vt, xt, range=mode, mlp=mlp)
        assert mlp.fallback_count() == n
        with threshold(bk, 1 << 14):
            lk = bk.logk(vt, xt, range=mode, mlp=mlp)
            assert mlp.fallback_count() == 0
            l2, dv, dx = bk.logk_dv_dx(vt, xt, grad_out=go, range=mode, mlp=mlp)
            plain = bk.logk(vt, xt)
            pl2, pdv, pdx = bk.logk_dv_dx(vt, xt, grad_out=go)
        assert torch.equal(lk, plain) and torch.equal(l2, pl2)
        assert torch.equal(dv, pdv) and torch.equal(dx, pdx)
        ref, rdv, rdx = oracle.logk(host(vt), host(xt), deriv=True)
        assert mixed(host(lk), ref).max() <= 1e-5
        g = host(go)
        assert mixed(host(dv), g * rdv).max() <= 1e-5 and mixed(host(dx), g * rdx).max() <= 1e-5
    finally:
        mlp.close()
