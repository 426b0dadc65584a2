#!/usr/bin/env python3
"""Benchmark of the regularized Stokes single layer on one MI355X.

A step is one full evaluation u = S^delta[f] at every node of the biconcave surface with
6 x 64 x 64 nodes (N = 24,576), SH force density, delta = 2h: spatial sort + packing,
pair kernel and per-target reduction, all through sl_eval, with inputs resident in HBM.
`value` is N^2 / t_step in Gpair/s for the headline precision (mixed by default); the
double-precision path, the 6 x 256 x 256 surface and the serving stream are reported beside
it.  Prints exactly one JSON line on stdout; progress goes to stderr.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_TFLOPS = {"fp64": 78.6, "mixed": 157.3}     # MI355X vector FP64 / FP32 (published)
FLOPS_FAR = 28                                   # plain Stokeslet pair
FLOPS_NEAR = 49                                  # regularized pair (erf, exp, rsqrt = 1 each)
RHO_EXACT64 = 6.9                                # s = 1 to double precision beyond this r/delta
PMC_FILE = os.path.join(ROOT, "profiles", "pmc_pair_kernel.json")
PAIR_SOURCES = ["paper_2310_13908_amd/csrc/sl_pair.hip", "paper_2310_13908_amd/csrc/sl_device.h"]


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def pair_kernel_sha() -> str:
    h = hashlib.sha256()
    for p in PAIR_SOURCES:
        h.update(open(os.path.join(ROOT, p), "rb").read())
    return h.hexdigest()[:16]


def count_near(X, delta, cuts, chunk=512):
    """Exact number of (target, source) pairs with r / delta < cut, for each cut (fp64 on the
    GPU, plain differences -- measurement bookkeeping, not part of the timed path)."""
    n = X.shape[0]
    out = {c: 0 for c in cuts}
    for i in range(0, n, chunk):
        d2 = (X[i:i + chunk, None, :] - X[None, :, :]).square_().sum(dim=-1)
        for c in cuts:
            out[c] += int((d2 < (c * delta) ** 2).sum().item())
        del d2
    return out


def time_steps(fn, steps, warmup):
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        fn()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / steps


def measure_precision(ctx, P, prob, tens, precision, steps, warmup):
    """ms per full evaluation, and the average pair-kernel duration from the library's events."""
    X, w, F = tens
    out = __import__("torch").empty((3, prob.N), dtype=__import__("torch").float64, device=X.device)
    fn = lambda: ctx.single_layer(X, w, F, prob.delta, precision=precision, out=out)
    for _ in range(warmup):
        fn()
    s0 = P.sl_get_stats(ctx.ptr)
    P.check(P.sl_set_param(ctx.ptr, P.SL_PARAM_KERNEL_TIMING, 1.0))
    t = time_steps(fn, steps, 0)
    P.check(P.sl_set_param(ctx.ptr, P.SL_PARAM_KERNEL_TIMING, 0.0))
    s1 = P.sl_get_stats(ctx.ptr)
    launches = s1.pair_launches - s0.pair_launches
    kern_ms = (s1.pair_ms - s0.pair_ms) / max(1, launches)
    return t * 1e3, kern_ms, out


def roofline(precision, pairs, near, kern_ms):
    flops = FLOPS_FAR * (pairs - near) + FLOPS_NEAR * near
    achieved = flops / (kern_ms * 1e-3) / 1e12
    peak = PEAK_TFLOPS[precision]
    traffic = None
    if os.path.exists(PMC_FILE):
        rec = json.load(open(PMC_FILE))
        entry = rec.get("kernels", {}).get(precision)
        if entry and rec.get("pair_kernel_sha") == pair_kernel_sha():
            traffic = entry["hbm_bytes_per_launch"]
    return {"bound": "alu", "achieved": round(achieved, 3), "peak": peak, "unit": "TFLOP/s",
            "frac": round(achieved / peak, 4), "traffic": traffic,
            "kernel_ms": round(kern_ms, 4), "flops_per_launch": flops,
            "flops_per_pair": {"far": FLOPS_FAR, "near": FLOPS_NEAR}, "near_pairs": near,
            "pairs": pairs}


def cpu_baseline(prob):
    """The oracle as it stands, on the host cores, over the whole workload (all targets)."""
    import oracle
    oracle.build(force=False)
    threads = oracle.max_threads()
    t0 = time.perf_counter()
    oracle.single_layer(prob.surface.X, prob.surface.w, prob.f, prob.delta)
    dt = time.perf_counter() - t0
    return {"value": round(prob.N ** 2 / dt / 1e9, 4), "unit": "Gpair/s", "cores": threads,
            "kind": "oracle", "seconds": round(dt, 3),
            "sample": f"all {prob.N} targets x {prob.N} sources of the same surface and density"}


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--precision", choices=["mixed", "fp64"], default="mixed")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true", help="skip the large-N and serving legs")
    ap.add_argument("--copy-bytes", type=int, default=0,
                    help="also run one device copy of this many bytes (PMC calibration)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: this build has no multi-GPU path (the sum would shard "
              "over targets after one all-gather of the sources); run with --gpus 1.",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_2310_13908_amd as P
    from capsule_inputs import workloads as W

    dev = torch.device("cuda", 0)
    ctx = P.Context(0)
    prob = W.c2()
    tens = tuple(torch.as_tensor(a, device=dev) for a in (prob.surface.X, prob.surface.w, prob.f))
    pairs = prob.N * prob.N
    log(f"[bench] workload c2: RBC 6x64x64, N={prob.N}, delta={prob.delta:.6g}")
    near = count_near(tens[0], prob.delta, [RHO_EXACT64, 5.0])

    res = {}
    for prec in ("fp64", "mixed"):
        ms, kern_ms, _ = measure_precision(ctx, P, prob, tens, prec, args.steps, args.warmup)
        near_p = near[RHO_EXACT64] if prec == "fp64" else near[5.0]
        res[prec] = {"ms_per_step": round(ms, 4), "gpair_s": round(pairs / (ms * 1e-3) / 1e9, 3),
                     "roofline": roofline(prec, pairs, near_p, kern_ms)}
        log(f"[bench] {prec}: {ms:.3f} ms/step  {res[prec]['gpair_s']:.1f} Gpair/s  "
            f"pair kernel {kern_ms:.3f} ms  {res[prec]['roofline']['frac'] * 100:.1f}% of peak")

    head = res[args.precision]
    other = "fp64" if args.precision == "mixed" else "mixed"
    line = {
        "metric": "Gpair/s regularized Stokeslet sum, FP32-mixed vs FP64; p50/p99 latency",
        "value": head["gpair_s"], "unit": "Gpair/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": head["ms_per_step"], "higher_is_better": True,
        "scaling": "strong", "vs_baseline": None,
        "dtype": "f32+f64" if args.precision == "mixed" else "f64",
        "data": "synthetic",
        "config": {"workload": "rbc_6x64x64_sh8", "N": prob.N, "delta": prob.delta, "mu": 1.0,
                   "precision": args.precision, "seed": W.SEED_C2,
                   "step": "sl_eval: sort + pack + pair kernel + reduction, all N targets"},
        "roofline": {k: head["roofline"][k] for k in
                     ("bound", "achieved", "peak", "unit", "frac", "traffic")},
        "roofline_detail": head["roofline"],
        other: res[other],
    }

    if not args.no_extras:
        p3 = W.c3()
        t3 = tuple(torch.as_tensor(a, device=dev) for a in (p3.surface.X, p3.surface.w, p3.f))
        big = {"workload": "rbc_6x256x256_sh8", "N": p3.N}
        for prec in ("fp64", "mixed"):
            ms, kern_ms, _ = measure_precision(ctx, P, p3, t3, prec, 3, 1)
            big[prec] = {"ms_per_step": round(ms, 3),
                         "gpair_s": round(p3.N ** 2 / (ms * 1e-3) / 1e9, 2),
                         "pair_kernel_ms": round(kern_ms, 3)}
            log(f"[bench] N={p3.N} {prec}: {ms:.2f} ms  {big[prec]['gpair_s']:.0f} Gpair/s")
        line["large_n"] = big
        del t3

    if args.copy_bytes:
        a = torch.empty(args.copy_bytes // 8, dtype=torch.float64, device=dev).fill_(1.0)
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        line["copy_calibration_bytes"] = args.copy_bytes

    if not args.no_cpu_baseline:
        log("[bench] cpu baseline: oracle on the host")
        line["cpu_baseline"] = cpu_baseline(prob)
    ctx.close()
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
