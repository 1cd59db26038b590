"""Benchmark: log K_v(x) evaluations per second on one MI355X.

Workload: the 2^24-pair scale workload (v ~ U[0, 50], x ~ 10^U[-3, 3], with 25 %
drawn from the hard bands |v - x| < 1 and v > 20, x < 0.1; seed 1), inputs
resident in HBM before timing.  Each path is timed over the whole batch at
128 bins:

    f32_mlp_fwd      FP32 bins on the learned bracket, Newton fallback (the
                     headline value: one step = one call over the batch)
    f32_mlp_fwd_bwd  the same with d/dv, d/dx log K times an upstream gradient
    f64_fwd          the plain method in FP64 (Newton bracket), log K
    f64_fwd_bwd
    f64_hess         log K with first and second derivatives, FP64
    f32_fwd          FP32 bins on the Newton bracket
    f32_fwd_bwd
    f32_hess
    gh_f32_fwd_bwd   per-set sums over 1024 sets x 65536 samples with gradients
    f64_logdk_1_1    d2K/dvdx with its own peak and bracket (bessel_logdk), FP64
    f32_mlp_table_fwd, f32_mlp_table_fwd_bwd
                     the learned bracket read from the network's bilinear table

The predictor is trained (20000 Adam steps on 2^20 Newton brackets) and its
margins calibrated before any timing.  Every launch runs on torch's current
stream, so the torch.cuda events around the timed region bracket exactly the
kernels.  Each path runs W warm-up calls, then untimed back-to-back calls for
--warm-seconds (the GPU's clock rises only under sustained load), then K timed
calls.  Prints ONE JSON line (rank 0).

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--warm-seconds S] [--nbins 128] [--no-cpu]
"""

from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import workloads  # noqa: E402

# Algorithmic VALU work per element, in lane-slots (one full-rate VALU
# instruction on one lane = 1 slot; an FP32 transcendental = 2, measured half
# rate; v_rcp_f64 = 4):  W(n) = (n + 1) * W_NODE + W_PRE, from the operation
# count of the formulation.  Per FP32 node: argument 1, conversion 1, exp2 2,
# widening 1, sum 1, u 1, linear part 1, cosh recurrence 1 (= 9); with d/dv and
# d/dx + r, t, w r, w u and two sums (= 15); second derivatives + 6 (= 21).
# Per FP64 node: 2 (cosh t - 1) as a product 1, argument 2 (v t - G advanced by
# one FMA, then the cosh term), exp 12 (clamp 1, reduction 4, degree-3
# polynomial 3, table index 1, table product 1, 2^k 2; the table read is an
# LDS load), sum 1, u 1, the two expm1 recurrences 2, re-anchoring 1.5
# (= 20.5), + 6 with d/dv and d/dx (t by addition, r, w r, w u, two sums),
# + 13 more for the second derivatives (cosh t - 1 from the product, six
# moments about the peak, two operations each).  W_PRE: peak (4 Newton steps)
# 100, the shift G in FP32 arithmetic 20, t1 50, t0 60, bin set-up 120, final
# log and reciprocal 50, loads 20.  Keyed by (dtype, derivative order): 0 log K, 1 with d/dv and d/dx, 2
# with the second derivatives too.
W_NODE = {("f32", 0): 9.0, ("f32", 1): 15.0, ("f32", 2): 21.0,
          ("f64", 0): 20.5, ("f64", 1): 26.5, ("f64", 2): 39.5}
W_PRE = 420.0
# Learned bracket: the network's VALU work (64 first-layer clamps, two per
# f16 conversion with its clamp bit, 32; 64 second-layer cubics, two per
# packed group of 4 instructions -- conversion with clamp, one FMA, two
# products -- 128; features 6, outputs 4; its three layers' 56 MFMAs per 64
# elements run on the matrix cores and are not counted) plus bracket 10, shift
# 35, bin set-up 120, check 10, final 50, loads 30.
W_NET = 170.0
W_MLP_PRE = W_NET + 255.0
# The same network read from its bilinear table: features 8, cell index 12,
# two 16-byte loads, 6 FMAs, in place of the network's VALU work.
W_TAB = 30.0
# Issue-slot equivalents per element of the network's MFMAs (896 busy cycles
# per wavefront / 4 cycles per wave instruction), reported beside the VALU
# fraction, not counted in W.
MFMA_SLOT_EQUIV = 224.0
W_TAB_PRE = W_TAB + 255.0

# MI355X vector issue peak: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz lane-slots/s
# (= the 78.6 TFLOP/s FP64 / unpacked-FP32 vector peak with an FMA as 2 FLOP).
PEAK_SLOTS = 256 * 4 * 16 * 2.4e9

# HBM bytes per element of the learned-range call (fused kernel + fallback)
# from rocprofv3 FETCH_SIZE (x2: a plain 256 MiB device copy reads back half
# its size on this counter) plus WRITE_SIZE, taken on the sources the kernels
# are compiled from (hashed below); reported only while they still match.
TRAFFIC = {"sources_sha256": "141c9de1d07d51691aa40454b409d37a16309dec1694136cec358933e0603d6c",
           # fused (65668 * 2 + 65623 KiB) + fallback (260 * 2 + 52 KiB) per 2^24 elements
           "bytes_per_elem": 12.056}
TRAFFIC_SOURCES = ("bessel_mlp.hip", "bessel_device.hpp", "bessel_internal.hpp", "bessel_learned.hpp",
                   "bessel_kernels.hip", "bessel_gh.hip")
# FP32 transcendental instructions (v_exp/log/rcp/sqrt_f32) per element, from
# the SQ_INSTS_VALU_TRANS_F32 counter per wavefront of 64 elements on the same
# sources (the FP64 paths' come from the FP32 bracket search; their
# exponentials and logarithms are FP64 software)
TRANS_F32_PER_ELEM = {"f32_fwd": 191, "f32_fwd_bwd": 192, "f32_hess": 192, "f64_fwd": 61, "f64_fwd_bwd": 61,
                      "f64_hess": 61, "f32_mlp_fwd": 144, "f32_mlp_fwd_bwd": 145, "f32_mlp_table_fwd": 144,
                      "f32_mlp_table_fwd_bwd": 145, "gh_f32_fwd_bwd": 166}


def kernel_sources_sha256() -> str:
    import hashlib
    csrc = os.path.join(ROOT, "paper_2108_11560_amd", "csrc")
    h = hashlib.sha256()
    for name in TRAFFIC_SOURCES:
        with open(os.path.join(csrc, name), "rb") as f:
            h.update(name.encode() + b"\0" + f.read())
    return h.hexdigest()


def alg_slots(dt: str, der: int, nbins: int) -> float:
    return (nbins + 1) * W_NODE[(dt, int(der))] + W_PRE


def alg_slots_mlp(grad: bool, nbins: int, fallback_rate: float, pre: float = W_MLP_PRE) -> float:
    """Per element of a learned-range call: the fused kernel's work (pre: its
    per-element work outside the bins), plus the Newton path for the fallback
    fraction."""
    return (nbins + 1) * W_NODE[("f32", int(grad))] + pre + fallback_rate * alg_slots("f32", grad, nbins)


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=20)
    p.add_argument("--warmup", type=int, default=3)
    p.add_argument("--warm-seconds", type=float, default=0.05,
                   help="after the warm-up calls, keep calling each path untimed for this long (sustained clock)")
    p.add_argument("--nbins", type=int, default=128)
    p.add_argument("--n", type=int, default=1 << 24)
    p.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline leg")
    p.add_argument("--cpu-seconds", type=float, default=12.0)
    p.add_argument("--mlp-steps", type=int, default=20000)
    p.add_argument("--copy-check", action="store_true",
                   help="also run a plain 256 MiB device copy (calibrates the FETCH_SIZE / WRITE_SIZE counters)")
    p.add_argument("--no-sweep", action="store_true", help="skip the batch-size sweep")
    p.add_argument("--no-configs", action="store_true",
                   help="skip the per-configuration block (plain 4096 FP64, differentiation 2^22, GH sums)")
    p.add_argument("--save-mlp", default=None, help="write the trained, calibrated predictor (.npz checkpoint with its provenance)")
    p.add_argument("--load-mlp", default=None,
                   help="use a predictor saved by --save-mlp instead of training one (for counter runs, "
                        "which serialise every dispatch)")
    return p.parse_args()


# The GPU raises its clock only under sustained load: a path timed right after
# an idle gap (host work, a synchronisation, another path's set-up) runs up to
# ~15 % slower for its first ~20 calls.  Each timed region therefore follows the
# W warm-up calls and then back-to-back untimed calls of the same path for at
# least --warm-seconds, so that it measures the sustained rate.
def time_path(fn, steps, warmup, warm_s=None):
    import torch
    warm_s = WARM_S if warm_s is None else warm_s
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    while time.perf_counter() - t0 < warm_s:
        for _ in range(4):
            fn()
        torch.cuda.synchronize()
    start, end = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    start.record()
    for _ in range(steps):
        fn()
    end.record()
    torch.cuda.synchronize()
    return start.elapsed_time(end) / steps  # ms per step


def graph_us_per_call(fn, calls: int = 50, replays: int = 20):
    """Microseconds per call when `calls` calls are captured in one HIP graph
    and the graph is replayed: the device-side cost without the per-call host
    launch overhead."""
    import torch
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        fn()
    torch.cuda.current_stream().wait_stream(s)
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        for _ in range(calls):
            fn()
    g.replay()
    torch.cuda.synchronize()
    start, end = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    start.record()
    for _ in range(replays):
        g.replay()
    end.record()
    torch.cuda.synchronize()
    return 1e3 * start.elapsed_time(end) / (replays * calls)


def cpu_baseline(v, x, v32, x32, gpu, budget_s):
    """The oracle (as it stands) on a bounded random sample, on the host cores.

    The same sample also gives each GPU path's largest mixed error (FP32 paths
    against the oracle at their FP32-rounded inputs)."""
    import oracle
    threads = oracle.default_threads()
    rng = np.random.default_rng(77)
    order = rng.permutation(v.size)
    done = 0
    chunk = 4096
    elapsed = 0.0  # oracle time on the FP64 sample only
    errs = {k: [] for k in gpu}
    while True:
        idx = order[done:done + chunk]
        t0 = time.perf_counter()
        ref64 = oracle.logk(v[idx], x[idx], nthreads=threads)
        elapsed += time.perf_counter() - t0
        done += idx.size
        ref32 = oracle.logk(v32[idx], x32[idx], nthreads=threads)
        for k, g in gpu.items():
            ref = ref64 if k == "f64" else ref32
            errs[k].append(np.abs(g[idx] - ref) / np.maximum(1.0, np.abs(ref)))
        if elapsed >= budget_s or done >= v.size:
            break
    errs = {k: np.concatenate(e) for k, e in errs.items()}
    return {
        "value": done / elapsed,
        "unit": "evals/s",
        "cores": threads,
        "kind": "oracle",
        "sample": f"{done} random pairs of the 2^24 scale workload, log K only, long-double adaptive quadrature",
    }, errs, done


WARM_S = 0.05


def err_stats(got, ref) -> dict:
    """Mixed error |got - ref| / max(1, |ref|): max, 99.9th percentile, median."""
    e = np.abs(np.asarray(got, np.float64) - ref) / np.maximum(1.0, np.abs(ref))
    return {"max": float(e.max()), "p99.9": float(np.quantile(e, 0.999)), "median": float(np.median(e))}


def oracle_timed(fn):
    """(result, seconds) of one oracle call on the host cores."""
    t0 = time.perf_counter()
    out = fn()
    return out, time.perf_counter() - t0


def per_config(bk, mlp, nb, steps, warmup, paths, dev):
    """One entry per workload configuration: the GPU path's throughput at its
    own size, its error against the oracle (max / p99.9 / median mixed error)
    on all or a stratified part of its elements, and the oracle's own rate on
    that part (the CPU baseline, host cores; a baseline only)."""
    import torch

    import oracle
    from oracle import gh_ref
    threads = oracle.default_threads()
    out = {}
    # plain method, FP64, 4096 pairs (seed 0), Newton bracket: every pair checked
    v, x = workloads.plain_pairs(4096, seed=0)
    vt, xt = torch.tensor(v, device=dev), torch.tensor(x, device=dev)
    ms = time_path(lambda: bk.logk(vt, xt, nbins=nb), steps, warmup)
    got = bk.logk(vt, xt, nbins=nb).cpu().numpy()
    ref, sec = oracle_timed(lambda: oracle.logk(v, x, nthreads=threads))
    out["plain-fp64-4096"] = {"n": 4096, "dtype": "f64", "us_per_call": 1e3 * ms, "evals_per_s": 4096 / (ms * 1e-3),
                              "err_vs_oracle": err_stats(got, ref), "oracle_elements": 4096,
                              "cpu_oracle_evals_per_s": 4096 / sec, "cpu_cores": threads}
    # differentiation, 2^22 pairs as the scale workload (seed 3), fwd + bwd with
    # upstream gradients (seed 13), FP32 and FP64; oracle on 2^13 stratified pairs
    n3 = 1 << 22
    v, x, strata = workloads.scale_pairs(n3, seed=3)
    go = workloads.upstream_grad(n3, seed=13)
    idx = workloads.stratified_subset(strata, 1 << 13, seed=11)
    entry = {"n": n3}
    for dt, tdt in (("f64", torch.float64), ("f32", torch.float32)):
        vt, xt, gt = (torch.tensor(a, dtype=tdt, device=dev) for a in (v, x, go))
        fn = lambda: bk.logk_dv_dx(vt, xt, grad_out=gt, nbins=nb)  # noqa: E731
        ms = time_path(fn, max(1, steps // 2), warmup)
        lk, dv, dx = (t.double().cpu().numpy()[idx] for t in fn())
        vs, xs = vt.double().cpu().numpy()[idx], xt.double().cpu().numpy()[idx]
        (rl, rv, rx), sec = oracle_timed(lambda: oracle.logk(vs, xs, deriv=True, nthreads=threads))
        g = gt.double().cpu().numpy()[idx]
        entry[dt] = {"ms": ms, "evals_per_s": n3 / (ms * 1e-3), "err_vs_oracle": {
            "logk": err_stats(lk, rl), "grad_v": err_stats(dv, g * rv), "grad_x": err_stats(dx, g * rx)}}
        entry["oracle_elements"] = int(idx.size)
        entry["cpu_oracle_evals_per_s"] = idx.size / sec
    entry["cpu_cores"] = threads
    out["diff-2^22"] = entry
    # GH-shaped per-set sums: 1024 sets x 65536 samples, fwd + bwd, FP32, with
    # the Newton bracket and with the network's table; the oracle sums every
    # set over the first 256 samples (GPU sums of the same sub-batch)
    lam, alpha, delta, mu, y, gs = workloads.gh_batch(1024, 65536, seed=5, grad_seed=15)
    f32 = lambda a: torch.tensor(a, dtype=torch.float32, device=dev)  # noqa: E731
    args = [f32(a) for a in (lam, alpha, delta, mu, y)]
    entry = {"sets": 1024, "samples": 65536}
    n5 = 1024 * 65536
    sub = [f32(a) for a in (lam, alpha, delta, mu, y[:256])]
    hl = lambda a: a.double().cpu().numpy()  # noqa: E731
    (ref, scale), sec = oracle_timed(lambda: gh_ref.gh_sums(*(hl(a) for a in sub), hl(f32(gs)), nthreads=threads,
                                                            with_scales=True))
    for name, kw in (("newton", {}), ("mlp_table", {"range": "mlp_table", "mlp": mlp})):
        ms = time_path(lambda: bk.gh_logk_sum(*args, grad_sum=f32(gs), nbins=nb, **kw), max(1, steps // 4),
                       max(1, warmup))
        got = [hl(t) for t in bk.gh_logk_sum(*sub, grad_sum=f32(gs), nbins=nb, **kw)]
        # per-set error of the sum and of each gradient relative to the summed
        # magnitudes of the terms (the natural scale of a sum's rounding)
        entry[name] = {"ms": ms, "evals_per_s": n5 / (ms * 1e-3), "err_vs_oracle_relative": {
            k: err_stats(np.asarray(got[i]) / scale[i], np.asarray(ref[i]) / scale[i])
            for i, k in enumerate(("sum", "d_lambda", "d_alpha", "d_delta", "d_mu"))}}
    entry["oracle_elements"] = 1024 * 256
    entry["cpu_oracle_evals_per_s"] = 1024 * 256 / sec
    entry["cpu_cores"] = threads
    out["gh-1024x65536"] = entry
    return out


def main():
    global WARM_S
    args = parse()
    WARM_S = args.warm_seconds
    if args.gpus != 1:
        print(json.dumps({"error": "the benchmark runs on one GPU; --gpus must be 1 (the elementwise path has no "
                                   "cross-GPU step: shard the batch, one process per GPU)"}))
        sys.exit(2)
    import torch

    import paper_2108_11560_amd as bk

    dev = torch.device("cuda:0")
    v64, x64, strata = workloads.scale_pairs(args.n, seed=1)
    go64 = workloads.upstream_grad(args.n, seed=13)
    V = {"f64": torch.tensor(v64, device=dev), "f32": torch.tensor(v64, dtype=torch.float32, device=dev)}
    X = {"f64": torch.tensor(x64, device=dev), "f32": torch.tensor(x64, dtype=torch.float32, device=dev)}
    GO = {"f64": torch.tensor(go64, device=dev), "f32": torch.tensor(go64, dtype=torch.float32, device=dev)}
    nb = args.nbins

    if args.copy_check:
        src = torch.ones(1 << 26, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    # learned range: train on the 2^20-sample training workload (labels = Newton
    # brackets), calibrate the two margins on a held-out set; not timed
    from paper_2108_11560_amd import mlp as M
    t_train = time.perf_counter()
    if args.load_mlp:
        mlp = M.RangeMLP.load_file(args.load_mlp)
        p = mlp.params()
        losses = np.zeros(0, dtype=np.float32)
        m1, m0, cal_rate = float(p[M.O_META + 4]), float(p[M.O_META + 5]), None
        args.mlp_steps = 0
    else:
        vtr, xtr, _ = workloads.scale_pairs(1 << 20, seed=4)
        mlp = M.RangeMLP(M.glorot_params(0))
        losses = mlp.train(torch.tensor(vtr, dtype=torch.float32, device=dev),
                           torch.tensor(xtr, dtype=torch.float32, device=dev),
                           steps=args.mlp_steps, batch=8192, lr=3e-3, lr_final=3e-5, seed=1)
        vca, xca, _ = workloads.scale_pairs(1 << 16, seed=8)
        m1, m0, cal_rate = M.calibrate_margins(mlp, torch.tensor(vca, dtype=torch.float32, device=dev),
                                               torch.tensor(xca, dtype=torch.float32, device=dev),
                                               target_fallback=0.001)
    if args.save_mlp:
        mlp.save(args.save_mlp)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t_train

    paths = {}
    for dt in ("f32", "f64"):
        fwd = lambda dt=dt: bk.logk(V[dt], X[dt], nbins=nb)  # noqa: E731
        fb = lambda dt=dt: bk.logk_dv_dx(V[dt], X[dt], grad_out=GO[dt], nbins=nb)  # noqa: E731
        ms_f = time_path(fwd, args.steps, args.warmup)
        ms_b = time_path(fb, args.steps, args.warmup)
        paths[f"{dt}_fwd"] = {"ms": ms_f, "evals_per_s": args.n / (ms_f * 1e-3)}
        paths[f"{dt}_fwd_bwd"] = {"ms": ms_b, "evals_per_s": args.n / (ms_b * 1e-3)}
        hs = lambda dt=dt: bk.logk_hess(V[dt], X[dt], nbins=nb)  # noqa: E731
        ms_h = time_path(hs, max(1, args.steps // 2), args.warmup)
        paths[f"{dt}_hess"] = {"ms": ms_h, "evals_per_s": args.n / (ms_h * 1e-3)}

    # general derivative, each integrand over its own bracket: orders (1, 1)
    dk = lambda: bk.logdk(V["f64"], X["f64"], 1, 1, nbins=nb, want_sign=False)  # noqa: E731
    ms_d = time_path(dk, max(1, args.steps // 4), max(1, args.warmup))
    paths["f64_logdk_1_1"] = {"ms": ms_d, "evals_per_s": args.n / (ms_d * 1e-3)}

    fwd = lambda: bk.logk(V["f32"], X["f32"], nbins=nb, range="mlp", mlp=mlp)  # noqa: E731
    fb = lambda: bk.logk_dv_dx(V["f32"], X["f32"], grad_out=GO["f32"], nbins=nb, range="mlp", mlp=mlp)  # noqa: E731
    ms_f = time_path(fwd, args.steps, args.warmup)
    fb_fwd = mlp.fallback_count()
    ms_b = time_path(fb, args.steps, args.warmup)
    fb_bwd = mlp.fallback_count()
    paths["f32_mlp_fwd"] = {"ms": ms_f, "evals_per_s": args.n / (ms_f * 1e-3), "fallback_rate": fb_fwd / args.n}
    paths["f32_mlp_fwd_bwd"] = {"ms": ms_b, "evals_per_s": args.n / (ms_b * 1e-3), "fallback_rate": fb_bwd / args.n}
    fwd = lambda: bk.logk(V["f32"], X["f32"], nbins=nb, range="mlp_table", mlp=mlp)  # noqa: E731
    fb = lambda: bk.logk_dv_dx(V["f32"], X["f32"], grad_out=GO["f32"], nbins=nb, range="mlp_table",  # noqa: E731
                               mlp=mlp)
    ms_tf = time_path(fwd, args.steps, args.warmup)
    fb_tf = mlp.fallback_count()
    ms_tb = time_path(fb, args.steps, args.warmup)
    fb_tb = mlp.fallback_count()
    paths["f32_mlp_table_fwd"] = {"ms": ms_tf, "evals_per_s": args.n / (ms_tf * 1e-3), "fallback_rate": fb_tf / args.n}
    paths["f32_mlp_table_fwd_bwd"] = {"ms": ms_tb, "evals_per_s": args.n / (ms_tb * 1e-3),
                                      "fallback_rate": fb_tb / args.n}
    mlp_info = {"train_steps": args.mlp_steps, "train_seconds": t_train,
                "final_loss": float(losses[-1]) if losses.size else None, "loaded_from": args.load_mlp,
                "margin_t1": m1, "margin_t0": m0, "calibration_fallback_rate": cal_rate}

    # generalised-hyperbolic-shaped per-set sums: 1024 sets x 65536 shared samples, fwd+bwd
    glam, galpha, gdelta, gmu, gy, ggs = (torch.tensor(a, dtype=torch.float32, device=dev)
                                          for a in workloads.gh_batch(1024, 65536, seed=5, grad_seed=15))
    gh = lambda: bk.gh_logk_sum(glam, galpha, gdelta, gmu, gy, grad_sum=ggs, nbins=nb)  # noqa: E731
    ms_g = time_path(gh, max(1, args.steps // 4), max(1, args.warmup))
    n_gh = glam.numel() * gy.numel()
    paths["gh_f32_fwd_bwd"] = {"ms": ms_g, "evals_per_s": n_gh / (ms_g * 1e-3), "elements": n_gh,
                               "alg_slots_per_elem": alg_slots("f32", True, nb),
                               "valu_frac": alg_slots("f32", True, nb) * n_gh / (ms_g * 1e-3) / PEAK_SLOTS}

    for key, p in paths.items():
        if key.startswith(("gh", "f64_logdk")):
            continue
        der = 2 if key.endswith("hess") else 1 if key.endswith("bwd") else 0
        if "mlp_table" in key:
            p["alg_slots_per_elem"] = alg_slots_mlp(der == 1, nb, p["fallback_rate"], pre=W_TAB_PRE)
        elif "mlp" in key:
            p["alg_slots_per_elem"] = alg_slots_mlp(der == 1, nb, p["fallback_rate"])
        else:
            p["alg_slots_per_elem"] = alg_slots(key[:3], der, nb)
        p["valu_frac"] = p["alg_slots_per_elem"] * p["evals_per_s"] / PEAK_SLOTS
    if TRAFFIC["sources_sha256"] == kernel_sources_sha256():
        for key, p in paths.items():
            if key in TRANS_F32_PER_ELEM:
                p["trans_f32_per_elem"] = TRANS_F32_PER_ELEM[key]
                p["trans_f32_per_s"] = TRANS_F32_PER_ELEM[key] * p["evals_per_s"]

    head = paths["f32_mlp_fwd"]
    achieved = head["alg_slots_per_elem"] * head["evals_per_s"]
    traffic = None
    if TRAFFIC["bytes_per_elem"] and TRAFFIC["sources_sha256"] == kernel_sources_sha256():
        traffic = TRAFFIC["bytes_per_elem"] * args.n
    # batch-size sweep in the paper's shape (Section 3.4: v = 10^{2r} - 1,
    # x = 10^{3r' - 1}): microseconds per call, kernels and launch included;
    # the *_graph_us entries replay 50 captured calls per launch (device-side cost)
    sweep = {"n": [], "f64_us": [], "f64_one_lane_us": [], "f64_graph_us": [], "f64_one_lane_graph_us": [],
             "f32_mlp_us": [], "f32_mlp_graph_us": [], "f32_mlp_table_graph_us": []}
    for n_s in () if args.no_sweep else (10, 100, 1000, 10000, 100000, 1000000):
        vs_, xs_ = workloads.paper_sweep(n_s)
        v64s, x64s = torch.tensor(vs_, device=dev), torch.tensor(xs_, device=dev)
        v32s, x32s = v64s.float(), x64s.float()
        reps = 200 if n_s <= 100000 else 20
        sweep["n"].append(n_s)
        sweep["f64_us"].append(1e3 * time_path(lambda: bk.logk(v64s, x64s, nbins=nb), reps, 5))
        sweep["f64_graph_us"].append(graph_us_per_call(lambda: bk.logk(v64s, x64s, nbins=nb)))
        prev = bk.set_split_threshold(0)
        sweep["f64_one_lane_us"].append(1e3 * time_path(lambda: bk.logk(v64s, x64s, nbins=nb), reps, 5))
        sweep["f64_one_lane_graph_us"].append(graph_us_per_call(lambda: bk.logk(v64s, x64s, nbins=nb)))
        bk.set_split_threshold(prev)
        sweep["f32_mlp_us"].append(1e3 * time_path(lambda: bk.logk(v32s, x32s, nbins=nb, range="mlp", mlp=mlp),
                                                   reps, 5))
        sweep["f32_mlp_graph_us"].append(graph_us_per_call(
            lambda: bk.logk(v32s, x32s, nbins=nb, range="mlp", mlp=mlp)))
        sweep["f32_mlp_table_graph_us"].append(graph_us_per_call(
            lambda: bk.logk(v32s, x32s, nbins=nb, range="mlp_table", mlp=mlp)))

    # the FP32 learned-range path against the plain FP64 method on the same batch
    speedup = {"fwd": paths["f32_mlp_fwd"]["evals_per_s"] / paths["f64_fwd"]["evals_per_s"],
               "fwd_bwd": paths["f32_mlp_fwd_bwd"]["evals_per_s"] / paths["f64_fwd_bwd"]["evals_per_s"]}
    # and against the same FP32 bins on the method's own (Newton) bracket: the
    # per-element network costs more than the bracket search it replaces on
    # this chip (< 1), the network read from its table less (> 1)
    vs_newton = {k: paths[f"f32_mlp{t}_{d}"]["evals_per_s"] / paths[f"f32_{d}"]["evals_per_s"]
                 for k, t, d in (("fwd", "", "fwd"), ("fwd_bwd", "", "fwd_bwd"),
                                 ("table_fwd", "_table", "fwd"), ("table_fwd_bwd", "_table", "fwd_bwd"))}
    # mixed error of the FP32 paths against the FP64 path, over the whole batch,
    # at the FP32-rounded inputs
    ref = bk.logk(V["f32"].double(), X["f32"].double(), nbins=nb)
    err_f64 = {}
    for key, out in (("f32", bk.logk(V["f32"], X["f32"], nbins=nb)),
                     ("f32_mlp", bk.logk(V["f32"], X["f32"], nbins=nb, range="mlp", mlp=mlp))):
        e = (out.double() - ref).abs() / ref.abs().clamp_min(1.0)
        sub = e[::16]
        err_f64[key] = {"max": float(e.max()), "p99": float(torch.quantile(sub, 0.99)),
                        "p99.9": float(torch.quantile(sub, 0.999)), "median": float(torch.quantile(sub, 0.5))}
    del ref
    roofline = {
        "bound": "alu",
        "kernel": f"k_logk_mlp<false,{nb}> (+ k_logk_fallback on the fallback fraction)",
        "achieved": achieved / 1e12,
        "peak": PEAK_SLOTS / 1e12,
        "unit": "T VALU lane-slots/s",
        "frac": achieved / PEAK_SLOTS,
        "traffic": traffic,
        "alg_slots_per_elem": head["alg_slots_per_elem"],
        # the network's 56 f16 MFMAs per wavefront keep the matrix core busy
        # 896 cycles, which the SIMD does not overlap with VALU issue: 224
        # issue-slot equivalents per element (SQ_VALU_MFMA_BUSY_CYCLES / 4)
        "mfma_slot_equiv_per_elem": MFMA_SLOT_EQUIV,
        "frac_incl_mfma_issue": achieved * (head["alg_slots_per_elem"] + MFMA_SLOT_EQUIV)
        / head["alg_slots_per_elem"] / PEAK_SLOTS,
    }

    line = {
        "metric": "log K_v(x) evals/s FP64 vs FP32+MLP-range (fwd, fwd+bwd) at rel err 1e-12/1e-5",
        "value": head["evals_per_s"],
        "unit": "evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["ms"],
        "higher_is_better": True,
        # a fixed batch, which more GPUs would split (one slice each)
        "scaling": "strong",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "scale-2^24", "n": args.n, "nbins": nb, "range": "mlp", "seed": 1,
                   "path": "f32 learned-range fwd"},
        "speedup_vs_f64": speedup,
        "speedup_vs_f32_newton": vs_newton,
        "batch_scaling": sweep,
        "err_vs_f64_path": err_f64,
        "paths": paths,
        "learned_range": mlp_info,
        "roofline": roofline,
        # the paper's own figure, for context only (another stack, another
        # machine, and a different workload: no ratio is formed with it)
        "paper_context": {"value": 2e6, "unit": "evals/s", "dtype": "f64",
                          "hardware": "TensorFlow 2.6, Intel Xeon W-2123 / NVIDIA TITAN RTX (timing device unstated)",
                          "note": "about 5 ms per call, flat from 10 to 1e4 elements (Section 3.4); 2e6 evals/s "
                                  "would follow at 1e4 elements"},
    }
    if not args.no_configs:
        line["configs"] = per_config(bk, mlp, nb, args.steps, args.warmup, paths, dev)
    if not args.no_cpu:
        gpu = {
            "f64": bk.logk(V["f64"], X["f64"], nbins=nb).cpu().numpy(),
            "f32": bk.logk(V["f32"], X["f32"], nbins=nb).double().cpu().numpy(),
            "f32_mlp": bk.logk(V["f32"], X["f32"], nbins=nb, range="mlp", mlp=mlp).double().cpu().numpy(),
        }
        base, errs, _ = cpu_baseline(v64, x64, V["f32"].double().cpu().numpy(), X["f32"].double().cpu().numpy(),
                                     gpu, args.cpu_seconds)
        line["cpu_baseline"] = base
        line["max_err_vs_oracle_on_sample"] = {k: float(e.max()) for k, e in errs.items()}
        line["err_vs_oracle_on_sample"] = {k: {"max": float(e.max()), "p99.9": float(np.quantile(e, 0.999)),
                                               "median": float(np.median(e))} for k, e in errs.items()}
        # the paper's accuracy measure (Section 3.1), log10(|Delta| / eps + 1)
        # with eps of the path's dtype and Delta the mixed error on log K
        line["paper_accuracy_measure_on_sample"] = {
            k: float(np.log10(float(e.max()) / float(np.finfo(np.float64 if k == "f64" else np.float32).eps) + 1.0))
            for k, e in errs.items()}
    else:
        line["cpu_baseline"] = None
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
