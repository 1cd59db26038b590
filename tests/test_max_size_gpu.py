"""The GPU path past 2^31 elements (through the C ABI, via the binding).

* Every launch indexes elements with 64 bits: FP32 forward and
  forward+backward and FP64 forward on the Newton bracket over 2^31 + 4 099
  pairs, checked against the oracle on the first and last 4 096 elements and
  4 096 drawn at random, and finite everywhere.
* The learned range keeps its failures on a worklist of 32-bit indices, so it
  accepts at most 2^31 - 2 elements: at that size its outputs, including
  fallbacks at indices above 2^30, match the oracle, and one element more is
  rejected before any work.

Inputs are drawn on the device by torch's seeded generator, so no 8 GiB array
passes through the host: v uniform on [0, 50] and x = 10^u with u uniform on
[-3, 3], the bulk stratum of the scale workload.  The oracle sees the same
FP32 values, widened.
"""

import math

import numpy as np
import pytest
import torch

import oracle
import workloads

pytestmark = pytest.mark.gpu

N_BIG = (1 << 31) + 4099
N_MLP = (1 << 31) - 2  # the learned range's limit (worklist count and indices in int32)
TOL32 = 1e-5


@pytest.fixture(scope="module")
def bk():
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a GPU")
    import paper_2108_11560_amd as m
    m.load()
    return m


@pytest.fixture(scope="module")
def big_pairs(bk):
    g = torch.Generator(device="cuda")
    g.manual_seed(2024)
    v = torch.empty(N_BIG, dtype=torch.float32, device="cuda").uniform_(0.0, 50.0, generator=g)
    x = torch.empty(N_BIG, dtype=torch.float32, device="cuda").uniform_(-3.0, 3.0, generator=g)
    x.mul_(math.log(10.0)).exp_()
    yield v, x
    del v, x
    torch.cuda.empty_cache()


def sample(n, seed):
    rng = np.random.default_rng(seed)
    return np.unique(np.concatenate([np.arange(4096), np.arange(n - 4096, n), rng.integers(0, n, 4096)]))


def gather(t, idx):
    return t[torch.as_tensor(idx, device=t.device)].double().cpu().numpy()


def mixed_err(got, ref):
    return np.abs(got - ref) / np.maximum(1.0, np.abs(ref))


def test_newton_past_2p31(bk, big_pairs):
    v, x = big_pairs
    idx = sample(N_BIG, 1)
    assert idx.max() == N_BIG - 1 and (idx >= (1 << 31)).sum() >= 4096
    vs, xs = gather(v, idx), gather(x, idx)
    ref, rdv, rdx = oracle.logk(vs, xs, deriv=True)

    lk = bk.logk(v, x, nbins=128)
    assert bool(torch.isfinite(lk).all())
    assert mixed_err(gather(lk, idx), ref).max() <= TOL32
    del lk
    torch.cuda.empty_cache()

    lk, dv, dx = bk.logk_dv_dx(v, x, nbins=128)
    assert bool(torch.isfinite(dv).all()) and bool(torch.isfinite(dx).all())
    assert mixed_err(gather(lk, idx), ref).max() <= TOL32
    assert mixed_err(gather(dv, idx), rdv).max() <= TOL32
    assert mixed_err(gather(dx, idx), rdx).max() <= TOL32
    del lk, dv, dx
    torch.cuda.empty_cache()


def test_newton_fp64_past_2p31(bk, big_pairs):
    # the FP64 kernels (their exponential reads a table in LDS) at the same size
    v32, x32 = big_pairs
    v, x = v32.double(), x32.double()
    idx = sample(N_BIG, 5)
    ref = oracle.logk(gather(v, idx), gather(x, idx))
    lk = bk.logk(v, x, nbins=128)
    assert bool(torch.isfinite(lk).all())
    assert mixed_err(gather(lk, idx), ref).max() <= 1e-12
    del v, x, lk
    torch.cuda.empty_cache()


def test_learned_range_at_its_limit(bk, big_pairs):
    from paper_2108_11560_amd import mlp as M
    v, x = big_pairs
    mlp = M.RangeMLP(M.glorot_params(0))
    try:
        vt, xt, _ = workloads.scale_pairs(1 << 18, seed=4)
        vt = torch.tensor(vt, dtype=torch.float32, device="cuda")
        xt = torch.tensor(xt, dtype=torch.float32, device="cuda")
        mlp.train(vt, xt, steps=3000, batch=8192, lr=3e-3, lr_final=1e-4, seed=1)
        vc, xc, _ = workloads.scale_pairs(1 << 16, seed=8)
        M.calibrate_margins(mlp, torch.tensor(vc, dtype=torch.float32, device="cuda"),
                            torch.tensor(xc, dtype=torch.float32, device="cuda"), target_fallback=0.001)

        vm, xm = v[:N_MLP], x[:N_MLP]
        # one element past the limit: an argument error, nothing launched
        with pytest.raises(bk.BesselError):
            bk.logk(v[:N_MLP + 1], x[:N_MLP + 1], nbins=128, range="mlp", mlp=mlp)

        lk = bk.logk(vm, xm, nbins=128, range="mlp", mlp=mlp)
        n_fb = mlp.fallback_count()
        assert 0 < n_fb <= 0.02 * N_MLP
        assert bool(torch.isfinite(lk).all())
        idx = sample(N_MLP, 2)
        ref = oracle.logk(gather(vm, idx), gather(xm, idx))
        assert mixed_err(gather(lk, idx), ref).max() <= TOL32

        # the fallbacks: the same set from bessel_range's flags, some of them
        # above 2^30, and their outputs (written by the fallback kernel) right
        *_, fb = bk.bessel_range(vm, xm, range="mlp", mlp=mlp, want_fallback=True)
        half = N_MLP // 2  # (torch's nonzero takes fewer than 2^31 - 1 elements)
        flagged = torch.cat([torch.nonzero(fb[:half]).squeeze(1), torch.nonzero(fb[half:]).squeeze(1) + half])
        del fb
        assert flagged.numel() == n_fb
        assert int(flagged.max()) >= (1 << 30)
        rng = np.random.default_rng(3)
        pick = flagged.cpu().numpy()
        pick = np.unique(np.concatenate([pick[-512:], rng.choice(pick, size=min(2048, pick.size), replace=False)]))
        ref = oracle.logk(gather(vm, pick), gather(xm, pick))
        assert mixed_err(gather(lk, pick), ref).max() <= TOL32
        del lk, flagged
        torch.cuda.empty_cache()
    finally:
        mlp.close()


def test_forced_fallback_at_the_limit(bk, big_pairs):
    # every element on the worklist (zero weights, t1 = e^{-30}): the fallback
    # kernel's grid-stride loop runs past 2^31 - stride and must not wrap
    from paper_2108_11560_amd import mlp as M
    v, x = big_pairs
    vm, xm = v[:N_MLP], x[:N_MLP]
    p = np.zeros(M.NPARAMS, dtype=np.float32)
    p[M.O_META:M.O_META + 6] = [1.0, 3.0, 0.0, 4.0, -30.0, 0.0]
    mlp = M.RangeMLP(p)
    try:
        out = bk.logk(vm, xm, nbins=128, range="mlp", mlp=mlp)
        assert mlp.fallback_count() == N_MLP
        newton = bk.logk(vm, xm, nbins=128)
        assert torch.equal(out, newton)
        del out, newton
        torch.cuda.empty_cache()
    finally:
        mlp.close()
