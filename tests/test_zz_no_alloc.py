"""bessel_gh_logk_sum_noalloc (partials in the library's static device array)
against bessel_gh_logk_sum (partials in a stream-ordered temporary), through
the C ABI.  Both run the same kernels in the same order, so the outputs must
agree bit for bit; two calls in a row, the second smaller, check that the
static array's leftovers from a larger call do not leak into a later one, and
one call at the array's full size (the GH workload, 1024 sets x 65536
samples) checks its bound."""

import ctypes

import numpy as np
import pytest
import torch

import workloads
from paper_2108_11560_amd import _lib

pytestmark = pytest.mark.gpu

MAX_BLOCKS = 1 << 18


@pytest.fixture(scope="module")
def lib():
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a GPU")
    return _lib.load()


def dev32(a):
    return torch.tensor(np.asarray(a, dtype=np.float32), device="cuda")


def call(lib, fn_name, sets, y, gs, nbins=128):
    n = sets[0].numel()
    outs = [torch.full((n,), float("nan"), dtype=torch.float32, device="cuda") for _ in range(5)]
    p = lambda t: ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p(0)  # noqa: E731
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    rc = getattr(lib, fn_name)(n, *(p(t) for t in sets), y.numel(), p(y), p(gs), *(p(o) for o in outs), nbins,
                               _lib.RANGE_NEWTON, ctypes.c_void_p(0), stream)
    assert rc == 0, (fn_name, rc, lib.bessel_last_error())
    torch.cuda.synchronize()
    return outs


def batch(nsets, nsamp, seed):
    lam, alpha, delta, mu, y, gs = workloads.gh_batch(nsets, nsamp, seed=seed, grad_seed=seed + 100)
    return [dev32(a) for a in (lam, alpha, delta, mu)], dev32(y), dev32(gs)


@pytest.mark.parametrize("first,second", [((64, 8192), (16, 1000)), ((300, 2000), (7, 257))])
def test_two_calls_second_smaller(lib, first, second):
    for k, (nsets, nsamp) in enumerate((first, second)):
        print(f"no_alloc: {nsets} sets x {nsamp} samples (call {k + 1})", flush=True)
        sets, y, gs = batch(nsets, nsamp, seed=40 + k)
        ref = call(lib, "bessel_gh_logk_sum", sets, y, gs)
        got = call(lib, "bessel_gh_logk_sum_noalloc", sets, y, gs)
        for r, g in zip(ref, got):
            assert bool(torch.isfinite(g).all())
            assert torch.equal(r, g)


def test_full_size_and_nbins(lib):
    # exactly MAX_BLOCKS records: 1024 sets x 256 chunks of 256 samples
    print("no_alloc: 1024 sets x 65536 samples", flush=True)
    sets, y, gs = batch(1024, 65536, seed=5)
    ref = call(lib, "bessel_gh_logk_sum", sets, y, gs)
    got = call(lib, "bessel_gh_logk_sum_noalloc", sets, y, gs)
    assert all(torch.equal(r, g) for r, g in zip(ref, got))
    # then a smaller call at another bin count, without the upstream gradient
    sets, y, _ = batch(33, 999, seed=7)
    ref = call(lib, "bessel_gh_logk_sum", sets, y, None, nbins=64)
    got = call(lib, "bessel_gh_logk_sum_noalloc", sets, y, None, nbins=64)
    assert all(torch.equal(r, g) for r, g in zip(ref, got))


def test_rejects_beyond_the_static_array(lib):
    sets, y, gs = batch(1025, 65536, seed=9)
    n = sets[0].numel()
    outs = [torch.zeros(n, dtype=torch.float32, device="cuda") for _ in range(5)]
    p = lambda t: ctypes.c_void_p(t.data_ptr())  # noqa: E731
    rc = lib.bessel_gh_logk_sum_noalloc(n, *(p(t) for t in sets), y.numel(), p(y), p(gs), *(p(o) for o in outs),
                                        128, _lib.RANGE_NEWTON, ctypes.c_void_p(0), ctypes.c_void_p(0))
    assert rc == -1
    assert b"static partials" in lib.bessel_last_error()
    torch.cuda.synchronize()
    assert all(bool((o == 0).all()) for o in outs)  # nothing was queued
