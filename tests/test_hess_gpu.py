"""GPU parity of the second derivatives of log K (bessel_logk_hess, through the
C ABI) against the oracle, and second-order autograd.

Tolerances (mixed error |got - ref| / max(1, |ref|)): the path's bars, FP64
1e-12 and FP32 1e-5, for log K and for the first and second derivatives.  The
FP64 second derivatives are variances and a covariance under the normalised
integrand (of t, t tanh(vt) and cosh t); the FP64 kernel forms them from
moments about the peak, so they keep the bar where the integrand is narrow
(large v with small x, or large x), where E[cosh^2 t] exceeds Var cosh t by up
to ~1e8.  In FP32 the sums are FP64 and the nodes' FP32 exponentials perturb
all sums alike, which leaves the raw differences at the FP32 bar.
"""

import numpy as np
import pytest
import torch

import oracle
import workloads

pytestmark = pytest.mark.gpu

TOL1 = {torch.float64: 1e-12, torch.float32: 1e-5}
TOL2 = {torch.float64: 1e-12, torch.float32: 1e-5}


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


def check_against_oracle(bk, v, x, dt, nbins=128):
    vt, xt = dev(v, dt), dev(x, dt)
    got = np.stack([host(o) for o in bk.logk_hess(vt, xt, nbins=nbins)], axis=1)
    ref = oracle.logk_hess(host(vt), host(xt))
    err = mixed(got, ref)
    assert err[:, :3].max() <= TOL1[dt], err[:, :3].max(axis=0)
    assert err[:, 3:].max() <= TOL2[dt], err[:, 3:].max(axis=0)
    return err


@pytest.mark.parametrize("dt", [torch.float64, torch.float32])
def test_plain_4096(bk, dt):
    v, x = workloads.plain_pairs(4096, seed=0)
    err = check_against_oracle(bk, v, x, dt)
    print(dt, "max mixed error per output", err.max(axis=0))


@pytest.mark.parametrize("dt", [torch.float64, torch.float32])
def test_scale_workload_sampled(bk, dt):
    # at full size the kernel runs on all 2^20 pairs; the oracle checks a
    # stratified sample
    v, x, strata = workloads.scale_pairs(1 << 20, seed=1)
    idx = workloads.stratified_subset(strata, 3 * 1024, seed=11)
    vt, xt = dev(v, dt), dev(x, dt)
    outs = bk.logk_hess(vt, xt)
    got = np.stack([host(o)[idx] for o in outs], axis=1)
    ref = oracle.logk_hess(host(vt)[idx], host(xt)[idx])
    err = mixed(got, ref)
    assert err[:, :3].max() <= TOL1[dt]
    assert err[:, 3:].max() <= TOL2[dt]
    # every element finite, the two variances non-negative
    for o in outs:
        assert torch.isfinite(o).all()
    assert (outs[3] >= 0).all() and (outs[4] >= 0).all()


@pytest.mark.parametrize("nbins", [64, 256, 100])
def test_bin_counts(bk, nbins):
    v, x = workloads.plain_pairs(1000, seed=3)
    check_against_oracle(bk, v, x, torch.float64, nbins=nbins)


def test_bessel_equation_full_batch(bk):
    """x^2 K'' + x K' - (x^2 + v^2) K = 0 on every element of 2^20 pairs."""
    v, x, _ = workloads.scale_pairs(1 << 20, seed=2)
    vt, xt = dev(v, torch.float64), dev(x, torch.float64)
    _, _, dx, _, dxx, _ = bk.logk_hess(vt, xt, want=(False, False, True, False, True, False))
    dx, dxx = host(dx), host(dxx)
    terms = np.stack([x ** 2 * dxx, x ** 2 * dx ** 2, x * dx, x ** 2, v ** 2])
    resid = x ** 2 * (dxx + dx ** 2) + x * dx - (x ** 2 + v ** 2)
    assert np.max(np.abs(resid) / np.abs(terms).max(axis=0)) <= 1e-11


@pytest.mark.parametrize("dt", [torch.float64, torch.float32])
def test_first_order_outputs_match_dv_dx_kernel(bk, dt):
    v, x, _ = workloads.scale_pairs(50000, seed=7)
    vt, xt = dev(v, dt), dev(x, dt)
    lk, dv, dx, *_ = bk.logk_hess(vt, xt)
    lk1, dv1, dx1 = bk.logk_dv_dx(vt, xt)
    assert torch.equal(lk, lk1) and torch.equal(dv, dv1) and torch.equal(dx, dx1)


def test_parity_in_v(bk):
    v, x = workloads.plain_pairs(2000, seed=9)
    vt, xt = dev(v, torch.float64), dev(x, torch.float64)
    P = bk.logk_hess(vt, xt)
    N = bk.logk_hess(-vt, xt)
    for k in (0, 2, 3, 4):
        assert torch.equal(P[k], N[k])
    for k in (1, 5):
        assert torch.equal(P[k], -N[k])
    Z = bk.logk_hess(torch.zeros_like(xt), xt)
    assert (Z[1] == 0).all() and (Z[5] == 0).all() and (Z[3] > 0).all()


def test_domain_and_empty(bk):
    nan, inf = float("nan"), float("inf")
    v = dev([nan, 1.0, 1.0, 1.0, 1.0, inf], torch.float64)
    x = dev([1.0, nan, -1.0, 0.0, inf, 2.0], torch.float64)
    out = [host(o) for o in bk.logk_hess(v, x)]
    assert np.isnan(out[0][:3]).all()
    assert out[0][3] == inf and out[0][4] == -inf and out[0][5] == inf
    for o in out[1:]:
        assert np.isnan(o).all()
    e = torch.empty(0, dtype=torch.float64, device="cuda")
    assert all(o.numel() == 0 for o in bk.logk_hess(e, e))


def test_finite_differences_of_first_derivatives(bk):
    v, x, strata = workloads.scale_pairs(1 << 14, seed=12)
    idx = workloads.stratified_subset(strata, 1024, seed=13)
    v, x = v[idx], x[idx]
    v = np.maximum(v, 0.05)  # keep v - h > 0
    vt, xt = dev(v, torch.float64), dev(x, torch.float64)
    _, _, _, dvv, dxx, dvx = (host(o) for o in bk.logk_hess(vt, xt))
    h = 1e-3

    def d1(vv, xx):
        _, a, b = bk.logk_dv_dx(dev(vv, torch.float64), dev(xx, torch.float64))
        return host(a), host(b)

    def rich(f, z, hz):
        return (4 * (f(z + hz / 2) - f(z - hz / 2)) / hz - (f(z + hz) - f(z - hz)) / (2 * hz)) / 3

    fd_vv = rich(lambda vv: d1(vv, x)[0], v, h)
    fd_xx = rich(lambda xx: d1(v, xx)[1], x, h * x)
    fd_vx = rich(lambda xx: d1(v, xx)[0], x, h * x)
    # differences of the GPU's own first derivatives: their ~1e-14 rounding
    # divided by the step bounds the check near 1e-10
    assert mixed(fd_vv, dvv).max() <= 1e-8
    assert mixed(fd_xx, dxx).max() <= 1e-8
    assert mixed(fd_vx, dvx).max() <= 1e-8


def test_hess_vjp_kernel(bk):
    from paper_2108_11560_amd import _lib
    import ctypes
    n = 1000
    g = torch.Generator(device="cpu").manual_seed(3)
    a, b, p, q, m = (torch.randn(n, generator=g, dtype=torch.float64).cuda() for _ in range(5))
    gv, gx = torch.empty_like(a), torch.empty_like(a)
    lib = bk.load()
    vp = lambda t: ctypes.c_void_p(t.data_ptr() if t is not None else 0)  # noqa: E731
    st = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    _lib.check(lib.bessel_hess_vjp(1, n, vp(a), vp(b), vp(p), vp(q), vp(m), vp(gv), vp(gx), st), "vjp")
    torch.testing.assert_close(gv, a * p + b * m, rtol=1e-15, atol=1e-15)
    torch.testing.assert_close(gx, a * m + b * q, rtol=1e-15, atol=1e-15)
    _lib.check(lib.bessel_hess_vjp(1, n, vp(None), vp(b), vp(None), vp(q), vp(m), vp(gv), vp(gx), st), "vjp")
    torch.testing.assert_close(gv, b * m, rtol=0, atol=0)
    torch.testing.assert_close(gx, b * q, rtol=0, atol=0)


def test_second_order_autograd(bk):
    v = (torch.rand(16, dtype=torch.float64, device="cuda") * 8 + 0.2).requires_grad_()
    x = (torch.rand(16, dtype=torch.float64, device="cuda") * 5 + 0.1).requires_grad_()
    f = lambda a, b: bk.log_bessel_k(a, b)  # noqa: E731
    assert torch.autograd.gradgradcheck(f, (v, x), eps=1e-6, atol=1e-6, rtol=1e-5)
    # the Hessian of sum log K is diagonal per element: compare with the kernel
    lk = bk.log_bessel_k(v, x).sum()
    gv, gx = torch.autograd.grad(lk, (v, x), create_graph=True)
    hvv, hvx = torch.autograd.grad(gv.sum(), (v, x), retain_graph=True)
    hxv, hxx = torch.autograd.grad(gx.sum(), (v, x))
    _, _, _, dvv, dxx, dvx = bk.logk_hess(v.detach(), x.detach())
    assert torch.equal(hvv, dvv) and torch.equal(hxx, dxx)
    assert torch.equal(hvx, dvx) and torch.equal(hxv, dvx)


@pytest.mark.parametrize("dt", [torch.float64, torch.float32])
def test_validated_domain(bk, dt):
    # across the validated domain (v up to 1e3 and down to 1e-8, x in
    # [1e-6, 1e5]); the FP64 second derivatives were at 1.2e-11 (d2/dvdx at
    # v ~ 1e3, x ~ 3e-4) when formed from raw moments
    v, x = workloads.domain_pairs(800, seed=61)
    err = check_against_oracle(bk, v, x, dt)
    print(dt, "max mixed error per output", err.max(axis=0))


@pytest.mark.parametrize("dt", [torch.float64, torch.float32])
@pytest.mark.parametrize("split", [False, True])
def test_large_x_corners(bk, dt, split):
    # the validated domain's large-x edge (x up to 1e6), where the bracket is
    # ~1e-2 wide and cosh t - 1 ~ 1e-5 across it: the FP64 moments of cosh t
    # are taken about cosh t_p - 1, the FP32 shift subtracts x exactly
    v = np.repeat([0.0, 0.5, 10.0, 100.0, 1e3], 3)
    x = np.tile([1e5, 3e5, 1e6], 5)
    prev = bk.set_split_threshold(1 << 20 if split else 0)
    try:
        err = check_against_oracle(bk, v, x, dt)
    finally:
        bk.set_split_threshold(prev)
    print(dt, "split" if split else "one lane", "max mixed error per output", err.max(axis=0))
