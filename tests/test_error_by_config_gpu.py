"""Error against the FP64 path (and of the FP64 path against the oracle) for
each workload configuration, printed as one line per configuration and held
to the bars: mixed error |got - ref| / max(1, |ref|) of 1e-12 (FP64 against
the oracle) and 1e-5 (FP32 against FP64).  For the per-set sums, the error is
relative to the sum of the magnitudes of the summed terms.

  plain-fp64-4096   FP64 log K against the oracle (all 4096), FP32 against FP64
  scale-2^24        FP32 (64/128/256 bins) against FP64 at 128 bins; FP64 at
                    64/128/256 bins against the oracle on a stratified sample
  diff-2^22         FP32 d/dv, d/dx (times an upstream gradient) against FP64
  learned-2^24      the learned range (per element and tabulated) against FP64
  gh-1024x65536     FP32 per-set sums and gradients against FP64 sums of the
                    FP64 path's log K and derivatives on the same pairs
"""

import numpy as np
import pytest
import torch

import oracle
import workloads

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def bk():
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a GPU")
    import paper_2108_11560_amd as mod
    mod.load()
    return mod


def mixed(got, ref):
    got, ref = got.double(), ref.double()
    return float(((got - ref).abs() / ref.abs().clamp_min(1.0)).max())


def dev(a, dt=torch.float64):
    return torch.tensor(np.asarray(a), dtype=dt, device="cuda")


def test_plain_fp64_4096(bk):
    v, x = workloads.plain_pairs(4096, seed=0)
    lk64 = bk.logk(dev(v), dev(x))
    ref = torch.tensor(oracle.logk(v, x), device="cuda")
    e64 = mixed(lk64, ref)
    v32, x32 = dev(v, torch.float32), dev(x, torch.float32)
    e32 = mixed(bk.logk(v32, x32), bk.logk(v32.double(), x32.double()))
    print(f"plain-fp64-4096: FP64 vs oracle {e64:.2e}; FP32 vs FP64 {e32:.2e}")
    assert e64 <= 1e-12 and e32 <= 1e-5


def test_scale_2p24(bk):
    v, x, strata = workloads.scale_pairs(1 << 24, seed=1)
    v32, x32 = dev(v, torch.float32), dev(x, torch.float32)
    ref32in = bk.logk(v32.double(), x32.double())
    out = [f"scale-2^24: FP32 vs FP64 at nbins {nb}: {mixed(bk.logk(v32, x32, nbins=nb), ref32in):.2e}"
           for nb in (64, 128, 256)]
    for o in out:
        assert float(o.split()[-1]) <= 1e-5
    idx = workloads.stratified_subset(strata, 1 << 12, seed=11)
    ref = torch.tensor(oracle.logk(v[idx], x[idx]), device="cuda")
    vi, xi = dev(v[idx]), dev(x[idx])
    for nb in (64, 128, 256):
        e = mixed(bk.logk(vi, xi, nbins=nb), ref)
        out.append(f"scale-2^24: FP64 vs oracle (stratified 4096) at nbins {nb}: {e:.2e}")
        assert e <= 1e-12
    print("\n".join(out))


def test_diff_2p22(bk):
    v, x, _ = workloads.scale_pairs(1 << 22, seed=3)
    go = workloads.upstream_grad(1 << 22, seed=13)
    v32, x32, g32 = dev(v, torch.float32), dev(x, torch.float32), dev(go, torch.float32)
    _, dv32, dx32 = bk.logk_dv_dx(v32, x32, grad_out=g32)
    _, dv64, dx64 = bk.logk_dv_dx(v32.double(), x32.double(), grad_out=g32.double())
    ev, ex = mixed(dv32, dv64), mixed(dx32, dx64)
    print(f"diff-2^22: FP32 vs FP64 go*d/dv {ev:.2e}, go*d/dx {ex:.2e}")
    assert ev <= 1e-5 and ex <= 1e-5


def test_learned_2p24(bk):
    from paper_2108_11560_amd import mlp as M
    vtr, xtr, _ = workloads.scale_pairs(1 << 20, seed=4)
    mlp = M.RangeMLP(M.glorot_params(0))
    mlp.train(dev(vtr, torch.float32), dev(xtr, torch.float32), steps=20000, batch=8192, lr=3e-3, lr_final=3e-5,
              seed=1)
    vca, xca, _ = workloads.scale_pairs(1 << 16, seed=8)
    M.calibrate_margins(mlp, dev(vca, torch.float32), dev(xca, torch.float32), target_fallback=0.001)
    v, x, _ = workloads.scale_pairs(1 << 24, seed=1)
    v32, x32 = dev(v, torch.float32), dev(x, torch.float32)
    ref = bk.logk(v32.double(), x32.double())
    e_mlp = mixed(bk.logk(v32, x32, range="mlp", mlp=mlp), ref)
    fb_mlp = mlp.fallback_count()
    e_tab = mixed(bk.logk(v32, x32, range="mlp_table", mlp=mlp), ref)
    fb_tab = mlp.fallback_count()
    print(f"learned-2^24: per-element network vs FP64 {e_mlp:.2e} (fallback {fb_mlp / v.size:.2e}); "
          f"table vs FP64 {e_tab:.2e} (fallback {fb_tab / v.size:.2e})")
    assert e_mlp <= 1e-5 and e_tab <= 1e-5
    mlp.close()


def test_gh_1024x65536(bk):
    lam, alpha, delta, mu, y, gs = workloads.gh_batch(1024, 65536, seed=5, grad_seed=15)
    f = lambda a: dev(a, torch.float32)  # noqa: E731
    s32, gl32, ga32, gd32, gm32 = bk.gh_logk_sum(f(lam), f(alpha), f(delta), f(mu), f(y), grad_sum=f(gs))
    # FP64 reference from the FP64 path on the same (FP32-rounded) parameters
    L, A, D, MU, Y, GS = (f(a).double() for a in (lam, alpha, delta, mu, y, gs))
    r = torch.sqrt(D[:, None] ** 2 + (Y[None, :] - MU[:, None]) ** 2)
    v = (L[:, None] - 0.5).expand_as(r).contiguous()
    x = (A[:, None] * r).contiguous()
    lk, dv, dx = bk.logk_dv_dx(v.reshape(-1), x.reshape(-1))
    lk, dv, dx = lk.view_as(r), dv.view_as(r), dx.view_as(r)
    ref = [lk.sum(1), GS * dv.sum(1), GS * (r * dx).sum(1), GS * (A[:, None] * D[:, None] / r * dx).sum(1),
           GS * (-A[:, None] * (Y[None, :] - MU[:, None]) / r * dx).sum(1)]
    scale = [lk.abs().clamp_min(1.0).sum(1), (GS[:, None] * dv).abs().sum(1).clamp_min(1.0),
             (GS[:, None] * r * dx).abs().sum(1).clamp_min(1.0),
             (GS[:, None] * A[:, None] * D[:, None] / r * dx).abs().sum(1).clamp_min(1.0),
             (GS[:, None] * A[:, None] * (Y[None, :] - MU[:, None]) / r * dx).abs().sum(1).clamp_min(1.0)]
    names = ["sum", "d/dlambda", "d/dalpha", "d/ddelta", "d/dmu"]
    errs = {}
    for name, got, rf, sc in zip(names, (s32, gl32, ga32, gd32, gm32), ref, scale):
        errs[name] = float(((got.double() - rf).abs() / sc).max())
    print("gh-1024x65536: FP32 vs FP64, relative to the summed magnitudes: "
          + ", ".join(f"{k} {e:.2e}" for k, e in errs.items()))
    assert max(errs.values()) <= 1e-5
