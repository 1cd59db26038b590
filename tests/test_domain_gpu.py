"""The GPU path at the corners of its validated domain and beyond, against
stored oracle values (tests/golden/domain_points.json, written by
make_domain_points.py, which calls only the oracle).

Validated (the bars of the path, mixed error, 128 bins): |v| <= 1e3 and
1e-6 <= x <= 1e6 in FP64 (1e-12), 1e-35 <= x <= 1e6 in FP32 (1e-5).  Beyond
(1e-35 <= x < 1e-6 in FP64) the results are finite and within the looser
bounds measured for them (FP64: 1e-8 on log K, 1e-4 on the derivatives).
Orders 1e4, 1e5 and 1e6 (tests/golden/large_order_points.json, same script,
x from 1e-30 to 1e6) hold the bars on log K and the first derivatives; the
FP64 second derivatives there hold 2e-9.  x below 1e-36 or above 1e36, |v|
above 1e6 and |v| above 1.2e38 x give NaN by convention.
"""

import json
import os

import numpy as np
import pytest
import torch

import oracle

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
PTS = json.load(open(os.path.join(HERE, "golden", "domain_points.json")))["points"]
LARGE = json.load(open(os.path.join(HERE, "golden", "large_order_points.json")))["points"]


@pytest.fixture(scope="module")
def bk():
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a GPU")
    import paper_2108_11560_amd as mod
    mod.load()
    return mod


def run(bk, dt, split, pts=PTS):
    v = np.array([p["v"] for p in pts])
    x = np.array([p["x"] for p in pts])
    ref = np.array([[p["logk"], p["dv"], p["dx"]] for p in pts])
    prev = bk.set_split_threshold(1 << 20 if split else 0)
    try:
        vt = torch.tensor(v, dtype=dt, device="cuda")
        xt = torch.tensor(x, dtype=dt, device="cuda")
        got = np.stack([t.double().cpu().numpy() for t in bk.logk_dv_dx(vt, xt)], axis=1)
    finally:
        bk.set_split_threshold(prev)
    err = np.abs(got - ref) / np.maximum(1.0, np.abs(ref))
    return v, x, got, err


@pytest.mark.parametrize("split", [False, True])
def test_fp64_domain(bk, split):
    v, x, got, err = run(bk, torch.float64, split)
    assert np.isfinite(got).all()
    inside = (x >= 1e-6) & (x <= 1e6)
    for i in np.flatnonzero(inside):
        assert err[i].max() <= 1e-12, (v[i], x[i], err[i])
    for i in np.flatnonzero(~inside):
        assert err[i, 0] <= 1e-8 and err[i, 1:].max() <= 1e-4, (v[i], x[i], err[i])


@pytest.mark.parametrize("split", [False, True])
def test_fp32_domain(bk, split):
    v, x, got, err = run(bk, torch.float32, split)
    assert np.isfinite(got).all()
    inside = x <= 1e6
    for i in np.flatnonzero(inside):
        assert err[i].max() <= 1e-5, (v[i], x[i], err[i])
    for i in np.flatnonzero(~inside):
        assert err[i, 0] <= 1e-5 and err[i, 1:].max() <= 1e-4, (v[i], x[i], err[i])


@pytest.mark.parametrize("dt", [torch.float64, torch.float32])
def test_below_range_is_nan(bk, dt):
    x = torch.tensor([1e-37, 5e-37, 2e-36], dtype=torch.float64).to(dt).cuda()
    v = torch.ones_like(x)
    lk, dv, dx = bk.logk_dv_dx(v, x)
    assert torch.isnan(lk[:2]).all() and torch.isnan(dv[:2]).all() and torch.isnan(dx[:2]).all()
    assert torch.isfinite(lk[2])


@pytest.mark.parametrize("dt", [torch.float64, torch.float32])
def test_beyond_search_range_is_nan(bk, dt):
    # x above 1e36, finite |v| above 1e6 and |v| above 1.2e38 x: NaN by
    # convention (x = +inf and |v| = +inf keep their limits); just inside,
    # finite (v / x = 1e38 at v = 1e3, x = 1e-35 is in the validated domain)
    v = torch.tensor([1.0, 1.0, 2e6, -2e6, 1e3, 1.0, float("inf"), 1.0, 9e5, -9e5, 1e3], dtype=torch.float64)
    x = torch.tensor([2e36, 1e38, 1.0, 1.0, 5e-36, float("inf"), 3.0, 5e35, 1.0, 1e-30, 1e-35], dtype=torch.float64)
    lk, dv, dx = (t.double().cpu().numpy() for t in bk.logk_dv_dx(v.to(dt).cuda(), x.to(dt).cuda()))
    assert np.isnan(lk[:5]).all() and np.isnan(dv[:5]).all() and np.isnan(dx[:5]).all()
    assert lk[5] == -np.inf and lk[6] == np.inf
    assert np.isfinite(lk[7:]).all() and np.isfinite(dv[7:]).all() and np.isfinite(dx[7:]).all()


# orders beyond the validated domain: log K and the first derivatives hold the
# path's bars; the FP64 second derivatives in x lose a few digits where the
# bracket is narrow (measured up to 3.7e-10 at v = 1e6)
BAR = {torch.float64: 1e-12, torch.float32: 1e-5}
BAR2 = {torch.float64: 2e-9, torch.float32: 1e-5}


@pytest.mark.parametrize("split", [False, True])
@pytest.mark.parametrize("dt", [torch.float64, torch.float32])
def test_large_orders(bk, dt, split):
    v, x, got, err = run(bk, dt, split, LARGE)
    assert np.isfinite(got).all()
    assert err.max() <= BAR[dt], (v[err.max(axis=1).argmax()], x[err.max(axis=1).argmax()], err.max())


@pytest.mark.parametrize("split", [False, True])
@pytest.mark.parametrize("dt", [torch.float64, torch.float32])
def test_large_orders_second_derivatives(bk, dt, split):
    v = np.array([p["v"] for p in LARGE])
    x = np.array([p["x"] for p in LARGE])
    ref = np.array([[p["d2v"], p["d2x"], p["dvx"]] for p in LARGE])
    prev = bk.set_split_threshold(1 << 20 if split else 0)
    try:
        out = bk.logk_hess(torch.tensor(v, dtype=dt).cuda(), torch.tensor(x, dtype=dt).cuda())
        got = np.stack([t.double().cpu().numpy() for t in out[3:]], axis=1)
    finally:
        bk.set_split_threshold(prev)
    # an FP32 output whose value exceeds the FP32 range is +-inf (d2/dx2 ~ v / x^2)
    over = np.abs(ref) > np.finfo(np.float32).max if dt == torch.float32 else np.zeros(ref.shape, bool)
    assert np.all(np.isinf(got[over]) & (np.sign(got[over]) == np.sign(ref[over])))
    err = np.abs(got - ref) / np.maximum(1.0, np.abs(ref))
    assert err[~over].max() <= BAR2[dt], err


@pytest.mark.parametrize("split", [False, True])
@pytest.mark.parametrize("dt", [torch.float64, torch.float32])
def test_search_range_limits_on_every_path(bk, dt, split):
    # the same limits on log K alone, the second derivatives and bessel_range
    v = torch.tensor([2e6, 1e3, 9e5, 1e3], dtype=torch.float64).to(dt).cuda()
    x = torch.tensor([1.0, 5e-36, 1.0, 1e-35], dtype=torch.float64).to(dt).cuda()
    prev = bk.set_split_threshold(1 << 20 if split else 0)
    try:
        lk = bk.logk(v, x).double().cpu().numpy()
        hs = [t.double().cpu().numpy() for t in bk.logk_hess(v, x)]
        rg = [t.double().cpu().numpy() for t in bk.bessel_range(v, x)]
    finally:
        bk.set_split_threshold(prev)
    for out in [lk, hs[0]] + rg:
        assert np.isnan(out[:2]).all() and np.isfinite(out[2:]).all()
    # inside, the derivatives are not NaN; in FP32 they may overflow where their
    # value does (d2/dx2 ~ v / x^2 = 1e73 at v = 1e3, x = 1e-35)
    for out in hs[1:]:
        assert np.isnan(out[:2]).all() and not np.isnan(out[2:]).any()


@pytest.mark.parametrize("dt", [torch.float64, torch.float32])
def test_large_order_brackets(bk, dt):
    # above |v| = 1e3 the ends start from the curvature bounds: the bracket
    # still contains the exact truncation set, and stays close to its width
    rng = np.random.default_rng(41)
    v = 10.0 ** rng.uniform(3.0, 6.0, 4096)
    x = 10.0 ** rng.uniform(-30.0, 6.0, 4096)
    # and flat peaks, x near v^2, where -g''(t_p) is small
    vf = 10.0 ** rng.uniform(3.0, 3.5, 512)
    v = np.concatenate([v, vf])
    x = np.concatenate([x, vf * vf * (1.0 + 10.0 ** rng.uniform(-7.0, -1.0, 512) * rng.choice([-1.0, 1.0], 512))])
    if dt == torch.float32:
        v, x = v.astype(np.float32).astype(np.float64), x.astype(np.float32).astype(np.float64)
    t0, t1, tp, G = (t.double().cpu().numpy() for t in bk.bessel_range(torch.tensor(v, dtype=dt).cuda(),
                                                                       torch.tensor(x, dtype=dt).cuda()))
    log_eps = float(np.log(np.finfo(np.float64 if dt == torch.float64 else np.float32).eps))
    tpe, Ge, t0e, t1e = oracle.range_exact(v, x, log_eps)
    assert np.all(t0 <= t0e * (1 + 1e-12)) and np.all(t1 >= t1e * (1 - 1e-12))
    ratio = (t1 - t0) / (t1e - t0e)
    assert np.quantile(ratio, 0.99) <= 2.5 and ratio.max() <= 3.0, (np.quantile(ratio, 0.99), ratio.max())
