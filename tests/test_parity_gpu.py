"""GPU parity of the HIP path (through the C ABI) against the CPU oracle.

Tolerances (mixed error |got - ref| / max(1, |ref|) on log K and on each
derivative):  FP64 1e-12, FP32 1e-5, the bars the method is held to.  FP32
results are compared with the oracle evaluated at the FP32-rounded inputs, so
input rounding is not counted as error.
"""

import numpy as np
import pytest
import torch

import oracle
import workloads

pytestmark = pytest.mark.gpu

TOL = {torch.float64: 1e-12, torch.float32: 1e-5}
LOG_EPS = {torch.float64: float(np.log(2.0 ** -52)), torch.float32: float(np.log(2.0 ** -23))}


@pytest.fixture(scope="module")
def bk():
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a GPU")
    import paper_2108_11560_amd as mod
    mod.load()
    return mod


def mixed(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return np.abs(a - b) / np.maximum(1.0, np.abs(b))


def to_dev(a, dt):
    return torch.tensor(np.asarray(a), dtype=dt, device="cuda")


def host(t):
    return t.double().cpu().numpy()


def oracle_at(v_t, x_t, deriv=False):
    """Oracle at exactly the values the GPU sees (FP32 inputs widened exactly)."""
    return oracle.logk(host(v_t), host(x_t), deriv=deriv)


@pytest.mark.parametrize("dt", [torch.float64, torch.float32])
@pytest.mark.parametrize("nbins", [64, 128, 256])
def test_plain_4096(bk, dt, nbins):
    v, x = workloads.plain_pairs(4096, seed=0)
    vt, xt = to_dev(v, dt), to_dev(x, dt)
    ref = oracle_at(vt, xt)
    got = host(bk.logk(vt, xt, nbins=nbins))
    assert mixed(got, ref).max() <= TOL[dt]


@pytest.mark.parametrize("dt", [torch.float64, torch.float32])
def test_derivatives_4096(bk, dt):
    v, x = workloads.plain_pairs(4096, seed=0)
    vt, xt = to_dev(v, dt), to_dev(x, dt)
    ref, rdv, rdx = oracle_at(vt, xt, deriv=True)
    lk, dv, dx = bk.logk_dv_dx(vt, xt, nbins=128)
    assert mixed(host(lk), ref).max() <= TOL[dt]
    assert mixed(host(dv), rdv).max() <= TOL[dt]
    assert mixed(host(dx), rdx).max() <= TOL[dt]


@pytest.mark.parametrize("dt", [torch.float64, torch.float32])
def test_scale_workload_sampled(bk, dt):
    # The full 2^24-pair workload in the launch configuration the benchmark times;
    # the oracle checks a stratified sample covering the hard bands.
    v, x, strata = workloads.scale_pairs(1 << 24, seed=1)
    idx = workloads.stratified_subset(strata, 1 << 13, seed=11)
    vt, xt = to_dev(v, dt), to_dev(x, dt)
    idx_t = torch.tensor(idx, device="cuda")
    for nbins in (64, 128, 256):
        out = bk.logk(vt, xt, nbins=nbins)
        assert bool(torch.isfinite(out).all())
        ref = oracle_at(vt[idx_t], xt[idx_t])
        assert mixed(host(out[idx_t]), ref).max() <= TOL[dt], nbins
    lk, dv, dx = bk.logk_dv_dx(vt, xt, nbins=128)
    ref, rdv, rdx = oracle_at(vt[idx_t], xt[idx_t], deriv=True)
    assert mixed(host(lk[idx_t]), ref).max() <= TOL[dt]
    assert mixed(host(dv[idx_t]), rdv).max() <= TOL[dt]
    assert mixed(host(dx[idx_t]), rdx).max() <= TOL[dt]


@pytest.mark.parametrize("n", [1, 63, 64, 65, 255, 256, 257, 1000, 4097])
def test_ragged_sizes(bk, n):
    v, x, _ = workloads.scale_pairs(n, seed=200 + n)
    for dt in (torch.float64, torch.float32):
        vt, xt = to_dev(v, dt), to_dev(x, dt)
        assert mixed(host(bk.logk(vt, xt, nbins=128)), oracle_at(vt, xt)).max() <= TOL[dt]


def test_empty(bk):
    e = torch.empty(0, dtype=torch.float64, device="cuda")
    assert bk.logk(e, e).numel() == 0
    lk, dv, dx = bk.logk_dv_dx(e, e)
    assert dv.numel() == 0


@pytest.mark.parametrize("nbins", [17, 48, 100, 129, 1000, 4096])
def test_generic_bin_counts(bk, nbins):
    v, x, _ = workloads.scale_pairs(2048, seed=300)
    vt, xt = to_dev(v, torch.float64), to_dev(x, torch.float64)
    got = host(bk.logk(vt, xt, nbins=nbins))
    err = mixed(got, oracle.logk(v, x))
    assert np.all(np.isfinite(got))
    if nbins >= 48:
        assert err.max() <= 1e-12
    else:
        assert err.max() <= 1e-3  # few bins: still a sane approximation


def test_two_bins_is_finite(bk):
    v, x, _ = workloads.scale_pairs(512, seed=301)
    got = host(bk.logk(to_dev(v, torch.float64), to_dev(x, torch.float64), nbins=2))
    assert np.all(np.isfinite(got))


@pytest.mark.parametrize("dt", [torch.float64, torch.float32])
def test_domain_conventions(bk, dt):
    nan, inf = float("nan"), float("inf")
    v = to_dev([nan, 1.0, 1.0, 1.0, 1.0, inf, -inf, 2.5, -2.5, 0.0], dt)
    x = to_dev([1.0, nan, -1.0, 0.0, inf, 2.0, 2.0, 3.0, 3.0, 3.0], dt)
    lk = host(bk.logk(v, x))
    assert np.isnan(lk[:3]).all()
    assert lk[3] == np.inf and lk[4] == -np.inf and lk[5] == np.inf and lk[6] == np.inf
    assert lk[7] == lk[8]  # K_{-v} = K_v, bitwise
    l2, dv, dx = bk.logk_dv_dx(v, x)
    dv, dx = host(dv), host(dx)
    assert np.isnan(dv[:7]).all() and np.isnan(dx[:7]).all()
    assert dv[7] == -dv[8] and dx[7] == dx[8]
    assert dv[9] == 0.0


def test_evenness_bitwise(bk):
    v, x, _ = workloads.scale_pairs(4096, seed=302)
    for dt in (torch.float64, torch.float32):
        vt, xt = to_dev(v, dt), to_dev(x, dt)
        assert torch.equal(bk.logk(vt, xt), bk.logk(-vt, xt))


@pytest.mark.parametrize("dt", [torch.float64, torch.float32])
def test_grad_out_fused(bk, dt):
    v, x, _ = workloads.scale_pairs(4096, seed=3)
    go = workloads.upstream_grad(4096, seed=13)
    vt, xt, gt = to_dev(v, dt), to_dev(x, dt), to_dev(go, dt)
    _, dv, dx = bk.logk_dv_dx(vt, xt)
    lk2, gv, gx = bk.logk_dv_dx(vt, xt, grad_out=gt)
    rel = 1e-15 if dt == torch.float64 else 2e-7
    assert np.all(np.abs(host(gv) - host(dv) * go) <= rel * np.abs(host(dv) * go) + 1e-300)
    assert np.all(np.abs(host(gx) - host(dx) * go) <= rel * np.abs(host(dx) * go) + 1e-300)


def test_autograd_function(bk):
    v, x, _ = workloads.scale_pairs(4096, seed=3)
    go = workloads.upstream_grad(4096, seed=13)
    for dt in (torch.float64, torch.float32):
        vt = to_dev(v, dt).requires_grad_(True)
        xt = to_dev(x, dt).requires_grad_(True)
        y = bk.log_bessel_k(vt, xt)
        y.backward(to_dev(go, dt))
        _, dv, dx = bk.logk_dv_dx(vt.detach(), xt.detach(), grad_out=to_dev(go, dt))
        assert torch.allclose(vt.grad, dv, rtol=1e-6 if dt == torch.float32 else 1e-14, atol=0)
        assert torch.allclose(xt.grad, dx, rtol=1e-6 if dt == torch.float32 else 1e-14, atol=0)
        assert torch.equal(y.detach(), bk.logk(vt.detach(), xt.detach()))


def test_gradcheck_fp64(bk):
    v, x, _ = workloads.scale_pairs(64, seed=303)
    vt = to_dev(v + 0.5, torch.float64).requires_grad_(True)  # keep v - eps away from 0
    xt = to_dev(x, torch.float64).requires_grad_(True)
    assert torch.autograd.gradcheck(lambda a, b: bk.log_bessel_k(a, b), (vt, xt), eps=1e-6, atol=1e-6, rtol=1e-6)


def test_finite_difference_1024(bk):
    # Central differences of the FP64 forward, step 1e-6, on the first 1024 pairs of
    # the differentiation workload (2^22 pairs drawn like the scale workload, seed 3).
    v, x, _ = workloads.scale_pairs(1 << 22, seed=3)
    v, x = v[:1024], x[:1024]
    h = 1e-6
    dt = torch.float64
    f = lambda a, b: host(bk.logk(to_dev(a, dt), to_dev(b, dt)))  # noqa: E731
    lk = f(v, x)
    _, dv, dx = bk.logk_dv_dx(to_dev(v, dt), to_dev(x, dt))
    dv, dx = host(dv), host(dx)
    # log K is even in v, so f(v - h) = f(|v - h|)
    fd_v = (f(v + h, x) - f(np.abs(v - h), x)) / (2 * h)
    hx = h * x
    fd_x = (f(v, x + hx) - f(v, x - hx)) / (2 * hx)
    # The forward carries rounding noise of a few eps times the largest term it
    # cancels (v t_p, x cosh t_p, |log K|); a difference quotient divides that
    # noise by the step.  Truncation O(h^2) is far below.
    tp, _, _, _ = oracle.range_exact(v, x, LOG_EPS[dt])
    noise = 1e-15 * (1.0 + np.abs(lk) + v * tp + x * np.cosh(tp))
    assert np.all(np.abs(dv - fd_v) <= 1e-8 * np.maximum(1.0, np.abs(dv)) + noise / h)
    assert np.all(np.abs(dx - fd_x) <= 1e-8 * np.maximum(1.0, np.abs(dx)) + noise / hx)


def test_finite_difference_richardson_1024(bk):
    # The same 1024 pairs with a step the rounding noise does not swamp:
    # central differences at h and h/2 combined by Richardson extrapolation
    # (truncation O(h^4) ~ 1e-12), h = 1e-3 in v and 1e-3 x in x.  The noise
    # term (a few eps of the largest cancelled term, over the step, times 3
    # for the extrapolation) is then ~1e-9 even at x ~ 1e3, so the bound
    # binds where the 1e-6 step above cannot.
    v, x, _ = workloads.scale_pairs(1 << 22, seed=3)
    v, x = v[:1024], x[:1024]
    dt = torch.float64
    f = lambda a, b: host(bk.logk(to_dev(a, dt), to_dev(b, dt)))  # noqa: E731
    lk = f(v, x)
    _, dv, dx = bk.logk_dv_dx(to_dev(v, dt), to_dev(x, dt))
    dv, dx = host(dv), host(dx)

    def rich(g, z, hz):
        d1 = (g(z + hz) - g(z - hz)) / (2 * hz)
        d2 = (g(z + hz / 2) - g(z - hz / 2)) / hz
        return (4 * d2 - d1) / 3

    h = 1e-3
    fd_v = rich(lambda a: f(np.abs(a), x), v, h)  # log K is even in v
    fd_x = rich(lambda b: f(v, b), x, h * x)
    tp, _, _, _ = oracle.range_exact(v, x, LOG_EPS[dt])
    noise = 1e-15 * (1.0 + np.abs(lk) + v * tp + x * np.cosh(tp))
    ev = np.abs(dv - fd_v) - 3 * noise / h
    ex = np.abs(dx - fd_x) - 3 * noise / (h * x)
    print("Richardson FD: max |dv - fd| %.2e, max |dx - fd| %.2e" % (np.abs(dv - fd_v).max(), np.abs(dx - fd_x).max()))
    assert np.all(ev <= 1e-9 * np.maximum(1.0, np.abs(dv)))
    assert np.all(ex <= 1e-9 * np.maximum(1.0, np.abs(dx)))


@pytest.mark.parametrize("dt", [torch.float64, torch.float32])
def test_range_invariants(bk, dt):
    v, x, strata = workloads.scale_pairs(1 << 16, seed=1)
    idx = workloads.stratified_subset(strata, 1 << 13, seed=12)
    vt, xt = to_dev(v[idx], dt), to_dev(x[idx], dt)
    t0, t1, tp, G = (host(a) for a in bk.bessel_range(vt, xt))
    tpe, Ge, t0e, t1e = oracle.range_exact(host(vt), host(xt), LOG_EPS[dt])
    # superset of the exact truncation set of Eq. (7)-(8)
    assert np.all(t0 <= t0e + 1e-12 * (1 + t0e))
    assert np.all(t1 >= t1e - 1e-12 * (1 + t1e))
    assert np.all((t0e > 0) | (t0 == 0))
    # peak value: G is g at the returned t_p (FP64 arithmetic for FP64, FP32
    # arithmetic for FP32, whose rounding is relative to the magnitudes of
    # log cosh(v t_p) and x cosh t_p), at most slightly below the true maximum
    scale = np.maximum(1.0, np.abs(Ge))
    if dt == torch.float64:
        rounding = 1e-13 * scale
    else:
        vd, xd = host(vt).astype(np.float64), host(xt).astype(np.float64)
        rounding = 1e-6 * (1.0 + np.abs(Ge) + vd * tpe + xd * np.cosh(tpe))
    assert np.all(G <= Ge + rounding)
    assert np.all(Ge - G <= 1e-3 * scale)
    assert np.all((tpe > 0) | (tp == 0))
    # tightness against the exact width
    ratio = (t1 - t0) / (t1e - t0e)
    assert np.quantile(ratio, 0.99) <= 1.6 and ratio.max() <= 3.0


def test_recurrence_self_consistency(bk):
    # K_{v+1} = K_{v-1} + (2v/x) K_v (the paper's Eq. (recu)) on GPU outputs alone.
    rng = np.random.default_rng(304)
    v = rng.uniform(1.0, 48.0, 8192)
    x = 10.0 ** rng.uniform(-3, 3, 8192)
    dt = torch.float64
    f = lambda a: host(bk.logk(to_dev(a, dt), to_dev(x, dt)))  # noqa: E731
    lm, l0, lp = f(v - 1), f(v), f(v + 1)
    rhs = np.logaddexp(lm, np.log(2 * v / x) + l0)
    assert mixed(lp, rhs).max() <= 2e-12


def test_deterministic(bk):
    v, x, _ = workloads.scale_pairs(1 << 18, seed=305)
    for dt in (torch.float64, torch.float32):
        vt, xt = to_dev(v, dt), to_dev(x, dt)
        assert torch.equal(bk.logk(vt, xt), bk.logk(vt, xt))
        a = bk.logk_dv_dx(vt, xt)
        b = bk.logk_dv_dx(vt, xt)
        assert all(torch.equal(p, q) for p, q in zip(a, b))


def test_paper_accuracy_grid(bk):
    # The paper's accuracy grid (Section 3.1): v = 10^{i/40} - 1, x = 10^{j/40 - 1}.
    v, x = workloads.accuracy_grid()
    ref = oracle.logk(v, x)
    got = host(bk.logk(to_dev(v, torch.float64), to_dev(x, torch.float64)))
    e = mixed(got, ref)
    assert e.max() <= 1e-12
    # the paper's metric log10(|Delta| / eps + 1), with Delta the mixed error of
    # log K (|log K| reaches ~400 on this grid, where one output ulp is ~26 eps)
    metric = np.log10(e / np.finfo(np.float64).eps + 1)
    assert np.median(metric) <= 1.0 and metric.max() <= 3.0  # at most 1000 eps (the bar, 1e-12, is ~4500 eps)
    ref32 = oracle.logk(v.astype(np.float32).astype(np.float64), x.astype(np.float32).astype(np.float64))
    got32 = host(bk.logk(to_dev(v, torch.float32), to_dev(x, torch.float32)))
    assert mixed(got32, ref32).max() <= 1e-5


def test_stream_ordering(bk):
    # A call on a side stream is ordered on that stream.
    v, x, _ = workloads.scale_pairs(1 << 16, seed=306)
    vt, xt = to_dev(v, torch.float64), to_dev(x, torch.float64)
    ref = bk.logk(vt, xt)
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        out = bk.logk(vt, xt)
    torch.cuda.current_stream().wait_stream(s)
    assert torch.equal(out, ref)


def test_paper_sweep_sizes(bk):
    # The paper's batch sweep shape (Section 3.4): sizes 10 .. 10^4, plus 10^6.
    for n in (10, 100, 1000, 10000, 1000000):
        v, x = workloads.paper_sweep(n)
        vt, xt = to_dev(v, torch.float64), to_dev(x, torch.float64)
        got = host(bk.logk(vt, xt))
        k = min(n, 2000)
        assert mixed(got[:k], oracle.logk(v[:k], x[:k])).max() <= 1e-12
