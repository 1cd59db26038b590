"""GPU parity of the general derivatives of K (bessel_logdk, through the C ABI):
each derivative integrand over its own peak and bracket (Section 4.1,
Eq. (13)), against the oracle's adaptive quadrature of the same integrand
(oracle.logdk, pinned by closed forms and recurrences on the CPU).

Tolerance: mixed error |got - ref| / max(1, |ref|) on log |D| of 1e-12 (F64)
and 1e-5 (F32), the bars of log K; signs exact.
"""

import numpy as np
import pytest
import torch

import oracle
import workloads

pytestmark = pytest.mark.gpu

TOL = {torch.float64: 1e-12, torch.float32: 1e-5}


@pytest.fixture(scope="module")
def bk():
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a GPU")
    import paper_2108_11560_amd as mod
    mod.load()
    return mod


def dev(a, dt):
    return torch.tensor(np.asarray(a), dtype=dt, device="cuda")


def host(t):
    return t.double().cpu().numpy()


def check(bk, v, x, a, b, dt, nbins=128):
    vt, xt = dev(v, dt), dev(x, dt)
    lg, sg = bk.logdk(vt, xt, a, b, nbins=nbins)
    ref, rs = oracle.logdk(host(vt), host(xt), a, b)
    lg, sg = host(lg), host(sg)
    assert np.array_equal(sg, rs), (a, b)
    fin = np.isfinite(ref)
    assert np.array_equal(lg[~fin], ref[~fin])
    err = np.abs(lg[fin] - ref[fin]) / np.maximum(1.0, np.abs(ref[fin]))
    assert err.max() <= TOL[dt], (a, b, float(err.max()))
    return err.max()


@pytest.mark.parametrize("a", range(4))
@pytest.mark.parametrize("b", range(4))
def test_scale_workload_f64(bk, a, b):
    # 1000 pairs: three full blocks of 256 and a ragged tail
    v, x, _ = workloads.scale_pairs(1000, seed=41)
    v = v * np.where(np.arange(1000) % 3 == 0, -1.0, 1.0)  # negative orders too
    check(bk, v, x, a, b, torch.float64)


@pytest.mark.parametrize("ab", [(8, 0), (0, 8), (5, 3), (8, 8), (1, 0), (0, 1), (2, 1)])
def test_validated_domain_high_orders(bk, ab):
    v, x = workloads.domain_pairs(600, seed=42)
    print(ab, check(bk, v, x, *ab, torch.float64))


@pytest.mark.parametrize("ab", [(0, 0), (1, 0), (0, 1), (2, 2), (4, 1)])
def test_f32(bk, ab):
    v, x, _ = workloads.scale_pairs(2000, seed=43)
    check(bk, workloads.to_f32(v), workloads.to_f32(x), *ab, torch.float32)


@pytest.mark.parametrize("nbins", [64, 100, 256])
def test_bin_counts(bk, nbins):
    v, x, _ = workloads.scale_pairs(700, seed=44)
    for ab in [(1, 0), (0, 2), (3, 3)]:
        check(bk, v, x, *ab, torch.float64, nbins=nbins)


def test_agrees_with_companion_sums(bk):
    # D_10 / K and D_01 / K are d/dv and d/dx of log K from bessel_logk_dv_dx
    # (f's bracket); compared in log space, mixed, as the oracle pins do
    v, x, _ = workloads.scale_pairs(4096, seed=45)
    vt, xt = dev(v, torch.float64), dev(x, torch.float64)
    lk, dv, dx = (host(t) for t in bk.logk_dv_dx(vt, xt))
    l00, _ = bk.logdk(vt, xt, 0, 0)
    assert np.max(np.abs(host(l00) - lk) / np.maximum(1, np.abs(lk))) <= 1e-13
    for (a, b), ref in (((1, 0), dv), ((0, 1), dx)):
        lg, sg = bk.logdk(vt, xt, a, b)
        lg, sg = host(lg), host(sg)
        nz = ref != 0
        assert np.all(np.sign(ref[nz]) == sg[nz])
        want = lk[nz] + np.log(np.abs(ref[nz]))
        assert np.max(np.abs(lg[nz] - want) / np.maximum(1, np.abs(want))) <= 1e-12


def test_conventions(bk):
    nan, inf = float("nan"), float("inf")
    v = np.array([nan, 1.0, 1.0, 1.0, inf, 0.0, 0.0, -1.5, 1.5, 2.0])
    x = np.array([1.0, -1.0, 0.0, inf, 1.0, 2.0, 2.0, 2.0, 2.0, 1e-37])
    for dt in (torch.float64, torch.float32):
        vt, xt = dev(v, dt), dev(x, dt)
        l1, s1 = (host(t) for t in bk.logdk(vt, xt, 1, 1))
        assert np.isnan(l1[0]) and np.isnan(s1[0]) and np.isnan(l1[1]) and np.isnan(s1[1])
        assert l1[2] == inf and l1[3] == -inf and l1[4] == inf
        assert l1[5] == -inf and s1[5] == 0.0  # odd order in v at v = 0
        assert s1[7] == 1.0 and s1[8] == -1.0 and l1[7] == l1[8]  # (-1)^b sign(v)
        assert np.isnan(l1[9])  # below x = 1e-36
        l2, s2 = (host(t) for t in bk.logdk(vt, xt, 2, 0))
        assert np.isfinite(l2[6]) and s2[6] == 1.0 and l2[7] == l2[8] and s2[7] == s2[8] == 1.0


def test_empty_and_no_sign(bk):
    e = torch.empty(0, dtype=torch.float64, device="cuda")
    lg, sg = bk.logdk(e, e, 2, 3)
    assert lg.numel() == 0 and sg.numel() == 0
    v, x, _ = workloads.scale_pairs(300, seed=46)
    vt, xt = dev(v, torch.float64), dev(x, torch.float64)
    a, _ = bk.logdk(vt, xt, 1, 2)
    b, none = bk.logdk(vt, xt, 1, 2, want_sign=False)
    assert none is None and torch.equal(a, b)


def test_full_size_sampled(bk):
    # the 2^24-pair scale workload in one launch; outputs sampled across the
    # strata against the oracle
    v, x, strata = workloads.scale_pairs(1 << 24, seed=1)
    vt, xt = dev(v, torch.float64), dev(x, torch.float64)
    lg, sg = bk.logdk(vt, xt, 1, 1)
    idx = workloads.stratified_subset(strata, 2048, seed=11)
    ref, rs = oracle.logdk(v[idx], x[idx], 1, 1)
    got = host(lg[torch.tensor(idx, device="cuda")])
    assert np.array_equal(host(sg[torch.tensor(idx, device="cuda")]), rs)
    assert np.max(np.abs(got - ref) / np.maximum(1, np.abs(ref))) <= 1e-12
    assert bool(torch.isfinite(lg).all())
