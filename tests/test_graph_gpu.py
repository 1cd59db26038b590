"""Capture of the Newton-path calls in a HIP graph (torch.cuda.CUDAGraph):
launch-bound small batches replay many calls with one launch.  The calls
launch only kernels on the current stream (no allocation, no memset), so they
can be captured; each replay is checked against the eager result, with eager
work and synchronisation between replays, and after the inputs change in
place."""

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
