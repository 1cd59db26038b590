"""Capture of library calls in a HIP graph (torch.cuda.CUDAGraph):
launch-bound small batches replay many calls with one launch.  The Newton
paths and bessel_logdk launch only kernels on the current stream (no
allocation, no memset); the learned-range paths do too once a first call has
built the predictor's operands, table and worklist.  Each replay is checked
against the eager result, with eager work and synchronisation between
replays, and after the inputs change in place."""

import numpy as np
import pytest
import torch

import workloads

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def bk():
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a GPU")
    import paper_2108_11560_amd as mod
    mod.load()
    return mod


@pytest.mark.parametrize("dt", [torch.float64, torch.float32])
@pytest.mark.parametrize("n", [1000, 100000])  # the split and the one-lane layouts
def test_capture_and_replay(bk, dt, n):
    v, x = workloads.paper_sweep(n, seed=41)
    v2, x2 = workloads.paper_sweep(n, seed=42)
    vt = torch.tensor(v, dtype=dt, device="cuda")
    xt = torch.tensor(x, dtype=dt, device="cuda")
    go = torch.tensor(workloads.upstream_grad(n, seed=43), dtype=dt, device="cuda")

    def calls():
        lk = bk.logk(vt, xt)
        _, dv, dx = bk.logk_dv_dx(vt, xt, grad_out=go, want_logk=False)
        h = bk.logk_hess(vt, xt)
        return lk, dv, dx, h[3], h[4], h[5]

    eager = calls()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        calls()  # warm-up on the side stream, as capture requires
    torch.cuda.current_stream().wait_stream(s)
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        static = calls()
    for rep in range(3):
        other = bk.logk(xt, xt)  # unrelated eager work between replays
        for t in static:
            t.fill_(float("nan"))
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        for a, b in zip(static, eager):
            assert torch.equal(a, b), rep
        assert torch.isfinite(other).all()
    # new inputs in place: the replay reads them
    vt.copy_(torch.tensor(v2, dtype=dt, device="cuda"))
    xt.copy_(torch.tensor(x2, dtype=dt, device="cuda"))
    fresh = calls()
    g.replay()
    torch.cuda.synchronize()
    for a, b in zip(static, fresh):
        assert torch.equal(a, b)


def _replay_matches(calls, inputs_update=None):
    eager = calls()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        calls()
    torch.cuda.current_stream().wait_stream(s)
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        static = calls()
    for rep in range(3):
        for t in static:
            t.fill_(float("nan"))
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        for a, b in zip(static, eager):
            assert torch.equal(a, b), rep
    if inputs_update is not None:
        inputs_update()
        fresh = calls()
        g.replay()
        torch.cuda.synchronize()
        for a, b in zip(static, fresh):
            assert torch.equal(a, b)


def test_capture_logdk(bk):
    v, x = workloads.paper_sweep(3000, seed=44)
    v2, _ = workloads.paper_sweep(3000, seed=45)
    vt = torch.tensor(v, device="cuda")
    xt = torch.tensor(x, device="cuda")

    def calls():
        a, sa = bk.logdk(vt, xt, 1, 0)
        b, _ = bk.logdk(vt, xt, 3, 2, nbins=100, want_sign=False)
        return a, sa, b

    _replay_matches(calls, lambda: vt.copy_(torch.tensor(v2, device="cuda")))


@pytest.mark.parametrize("mode", ["mlp", "mlp_table"])
def test_capture_learned_range(bk, mode):
    # after a warm-up call (operands, table and worklist in place) a
    # learned-range call launches only kernels: counter reset, fused pass and
    # the persistent fallback, whose trip count it reads on the device
    from paper_2108_11560_amd import mlp as M
    mlp = M.RangeMLP(M.glorot_params(11, margins=(0.05, 0.05)))
    v, x, _ = workloads.scale_pairs(20000, seed=46)
    v2, _, _ = workloads.scale_pairs(20000, seed=47)
    vt = torch.tensor(v, dtype=torch.float32, device="cuda")
    xt = torch.tensor(x, dtype=torch.float32, device="cuda")

    def calls():
        lk = bk.logk(vt, xt, range=mode, mlp=mlp)
        _, dv, dx = bk.logk_dv_dx(vt, xt, range=mode, mlp=mlp, want_logk=False)
        return lk, dv, dx

    _replay_matches(calls, lambda: vt.copy_(torch.tensor(v2, dtype=torch.float32, device="cuda")))
    mlp.close()
