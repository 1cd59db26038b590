"""The GPU path at the corners of its validated domain and beyond, against
stored oracle values (tests/golden/domain_points.json, written by
make_domain_points.py, which calls only the oracle).

Validated (the bars of the path, mixed error, 128 bins): |v| <= 1e3 and
1e-6 <= x <= 1e6 in FP64 (1e-12), 1e-35 <= x <= 1e6 in FP32 (1e-5).  Beyond
(1e-35 <= x < 1e-6 in FP64) the results are finite and within the looser
bounds measured for them (FP64: 1e-8 on log K, 1e-4 on the derivatives).
Orders 1e4, 1e5 and 1e6 (tests/golden/large_order_points.json, same script)
are finite and within the bounds measured for them, which grow with v.  x
below 1e-36 or above 1e36, |v| above 1e6 and |v| above 1.2e38 x give NaN by
convention.
"""

import json
import os

import numpy as np
import pytest
import torch

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


# mixed-error bounds at orders beyond the validated domain (log K, derivatives):
# the validated bars at 1e4, and about ten times the largest errors measured at
# these points at 1e5 (2.6e-7, 5.4e-4) and 1e6 (4.1e-6, 3.1e-3), both dtypes
LARGE_BOUNDS = {
    torch.float64: {1e4: (1e-12, 1e-12), 1e5: (2e-6, 5e-3), 1e6: (4e-5, 3e-2)},
    torch.float32: {1e4: (1e-5, 1e-5), 1e5: (2e-6, 5e-3), 1e6: (4e-5, 3e-2)},
}


@pytest.mark.parametrize("split", [False, True])
@pytest.mark.parametrize("dt", [torch.float64, torch.float32])
def test_large_orders(bk, dt, split):
    v, x, got, err = run(bk, dt, split, LARGE)
    assert np.isfinite(got).all()
    for i in range(v.size):
        b0, b1 = LARGE_BOUNDS[dt][v[i]]
        assert err[i, 0] <= b0 and err[i, 1:].max() <= b1, (v[i], x[i], err[i])


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
