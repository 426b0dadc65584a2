#!/usr/bin/env python3
"""Benchmark of the regularized Stokes single layer on one MI355X.

A step is one full evaluation u = S^delta[f] at every node of the biconcave surface with
6 x 256 x 256 nodes (N = 393,216; 1.55e11 pairs), SH force density, delta = 2h: spatial sort +
packing, pair kernel and per-target reduction, all through sl_eval, with inputs resident in HBM.
`value` is N^2 / t_step in Gpair/s for the headline precision (mixed by default); the
double-precision path, the 6 x 64 x 64 surface, the per-patch delta, the upsampling step and the
serving streams are reported beside it.  Prints exactly one JSON line on stdout; progress goes to
stderr.
"""
from __future__ import annotations

import argparse
import hashlib
import re
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
COPY_BYTES_PMC = 1 << 30                         # the calibration copy of the PMC passes
PAIR_SOURCES = ["paper_2310_13908_amd/csrc/sl_pair.hip", "paper_2310_13908_amd/csrc/sl_device.h",
                "paper_2310_13908_amd/csrc/sl_internal.h",
                "paper_2310_13908_amd/csrc/sl_smoothing_coeffs.h"]


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def code_text(src: str) -> str:
    """C++ source without comments and blank space: what the compiler sees of it."""
    src = re.sub(r"/\*.*?\*/", " ", src, flags=re.S)
    src = re.sub(r"//[^\n]*", " ", src)
    return " ".join(src.split())


def pair_kernel_sha() -> str:
    """Hash of the pair kernel's code (comments and layout excluded): the PMC traffic stored
    under profiles/ is reported only while it still matches."""
    h = hashlib.sha256()
    for p in PAIR_SOURCES:
        h.update(code_text(open(os.path.join(ROOT, p)).read()).encode())
    return h.hexdigest()[:16]


def count_near(X, delta, cuts, chunk=256):
    """Exact number of (target, source) pairs with r / delta < cut, for each cut (fp64 on the
    GPU, plain differences -- measurement bookkeeping, not part of the timed path)."""
    n = X.shape[0]
    Xt = X.t().contiguous()
    out = {c: 0 for c in cuts}
    for i in range(0, n, chunk):
        d2 = (X[i:i + chunk, 0:1] - Xt[0:1, :]).square_()
        d2 += (X[i:i + chunk, 1:2] - Xt[1:2, :]).square_()
        d2 += (X[i:i + chunk, 2:3] - Xt[2:3, :]).square_()
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
    """ms per full evaluation (steps timed back to back), and the average pair-kernel duration
    from the events the library records around its launch (a second pass: the events themselves
    add a few microseconds per evaluation, so they stay out of the timed steps)."""
    import torch
    X, w, F = tens
    out = torch.empty((3, prob.N), dtype=torch.float64, device=X.device)
    fn = lambda: ctx.single_layer(X, w, F, prob.delta, precision=precision, out=out)
    t = time_steps(fn, steps, warmup)
    s0 = P.sl_get_stats(ctx.ptr)
    P.check(P.sl_set_param(ctx.ptr, P.SL_PARAM_KERNEL_TIMING, 1.0))
    n_timed = max(3, min(steps, 20))
    time_steps(fn, n_timed, 0)
    P.check(P.sl_set_param(ctx.ptr, P.SL_PARAM_KERNEL_TIMING, 0.0))
    s1 = P.sl_get_stats(ctx.ptr)
    launches = max(1, s1.pair_launches - s0.pair_launches)
    kern_ms = (s1.pair_ms - s0.pair_ms) / launches
    return t * 1e3, kern_ms, out


def measure_headline(ctx, P, prob, tens, precision, steps, warmup, reps=30):
    """The timed region: `steps` evaluations back to back, with the HIP events that the library
    records around its pair-kernel launch on the caller's stream (the kernel's average duration
    over exactly these launches).  Then `reps` evaluations one at a time, each between two events
    on the same stream, for the median."""
    import torch
    X, w, F = tens
    out = torch.empty((3, prob.N), dtype=torch.float64, device=X.device)
    fn = lambda: ctx.single_layer(X, w, F, prob.delta, precision=precision, out=out)
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    s0 = P.sl_get_stats(ctx.ptr)
    P.check(P.sl_set_param(ctx.ptr, P.SL_PARAM_KERNEL_TIMING, 1.0))
    t0 = time.perf_counter()
    for _ in range(steps):
        fn()
    torch.cuda.synchronize()
    t = (time.perf_counter() - t0) / steps
    P.check(P.sl_set_param(ctx.ptr, P.SL_PARAM_KERNEL_TIMING, 0.0))
    s1 = P.sl_get_stats(ctx.ptr)
    launches = s1.pair_launches - s0.pair_launches
    kern_ms = (s1.pair_ms - s0.pair_ms) / max(1, launches)
    per = []
    cur = torch.cuda.current_stream()
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(cur)
        fn()
        e1.record(cur)
        e1.synchronize()
        per.append(e0.elapsed_time(e1))
    per.sort()
    return t * 1e3, kern_ms, int(launches), per[len(per) // 2], out


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform
    return platform.processor() or "unknown"


def cpu_baseline_sampled(prob, idx, idx_one):
    """The oracle as it stands on the host cores: all threads on the sampled targets `idx` (every
    source for each), and one thread on the first targets `idx_one`.  Returns the baseline record
    and the all-thread result (the reference for eps on those targets)."""
    import oracle
    oracle.build(force=False)
    X = prob.surface.X
    threads = oracle.max_threads()
    t0 = time.perf_counter()
    ref = oracle.single_layer(X, prob.surface.w, prob.f, prob.delta, targets=X[idx])
    dt = time.perf_counter() - t0
    t1 = time.perf_counter()
    oracle.single_layer(X, prob.surface.w, prob.f, prob.delta, targets=X[idx_one], nthreads=1)
    dt1 = time.perf_counter() - t1
    rate = len(idx) * prob.N / dt / 1e9
    rate1 = len(idx_one) * prob.N / dt1 / 1e9
    rec = {"value": round(rate, 5), "unit": "Gpair/s", "cores": threads, "kind": "oracle",
           "sample": f"{len(idx)} sampled targets x all {prob.N} sources of the same surface and "
                     f"density ({len(idx) * prob.N:.3g} pairs, {dt:.1f} s)",
           "cpu_model": cpu_model(), "seconds": round(dt, 3),
           "full_evaluation_s_extrapolated": round(prob.N * prob.N / (rate * 1e9), 1),
           "one_core": {"value": round(rate1, 5), "unit": "Gpair/s", "cores": 1,
                        "seconds": round(dt1, 3),
                        "sample": f"{len(idx_one)} of those targets x all {prob.N} sources"}}
    return rec, ref


def resident(dev, X, w, f):
    """Inputs resident in HBM in the library's structure-of-arrays layout: X and f are (N, 3)
    views of contiguous (3, N) tensors, so the binding passes them without a copy."""
    import numpy as np
    import torch
    soa = lambda a: torch.as_tensor(np.ascontiguousarray(np.asarray(a, dtype=np.float64).T), device=dev).t()
    return soa(X), torch.as_tensor(np.asarray(w, dtype=np.float64), device=dev), soa(f)


def patch_delta_leg(P, ctx, prob, tens, log, steps=20, warmup=3):
    """The same C2 workload with the paper's default regularization, delta = C delta*_i per
    patch (Sec. 3.4, eq. (regparam), C = 1): a step is the device pre-pass (sl_patch_delta)
    plus sl_eval with the per-target delta; every target against the oracle with the oracle's
    delta."""
    import numpy as np
    import torch
    import oracle
    X, w, F = tens
    n = prob.surface.n
    D = torch.empty(prob.N, dtype=torch.float64, device=X.device)
    out = torch.empty((3, prob.N), dtype=torch.float64, device=X.device)
    dref = oracle.patch_delta(prob.surface.X, n)
    t0 = time.perf_counter()
    ref = oracle.single_layer(prob.surface.X, prob.surface.w, prob.f, 0.0, delta_tgt=dref)
    log(f"[bench] per-patch delta: oracle in {time.perf_counter() - t0:.1f} s")
    per = dref.reshape(6, -1)[:, 0]
    res = {"workload": "rbc_6x64x64_sh8, delta = delta*_i per patch (C = 1)",
           "delta_star_min": float(per.min()), "delta_star_max": float(per.max()),
           "delta_2h": prob.delta}
    # the pre-pass alone
    pre = time_steps(lambda: ctx.patch_delta(X, n, out=D), steps, warmup)
    res["pre_pass_us"] = round(pre * 1e6, 2)
    res["delta_bit_exact"] = bool(np.array_equal(D.cpu().numpy(), dref))
    for prec in ("fp64", "mixed"):
        def step():
            ctx.patch_delta(X, n, out=D)
            ctx.single_layer(X, w, F, 0.0, delta_tgt=D, precision=prec, out=out)
        t = time_steps(step, steps, warmup)
        e = rel_inf(out.t().cpu().numpy(), ref)
        res[prec] = {"ms_per_step": round(t * 1e3, 4),
                     "gpair_s": round(prob.N ** 2 / t / 1e9, 2), "eps_vs_oracle": e}
        log(f"[bench] per-patch delta {prec}: {t * 1e3:.3f} ms/step  "
            f"{res[prec]['gpair_s']:.0f} Gpair/s  eps {e:.2e}")
    log(f"[bench] per-patch delta: pre-pass {res['pre_pass_us']:.1f} us, bit-exact "
        f"{res['delta_bit_exact']}, delta* in [{res['delta_star_min']:.4g}, "
        f"{res['delta_star_max']:.4g}] vs 2h = {prob.delta:.4g}")
    return res


def upsample_leg(P, ctx, dev, log, steps=3, warmup=1):
    """The paper's production form of the sum (Sec. 3.4, "Upsampling"): u = I_d S[I_u f] with a
    4x spline upsampling per patch, delta* on the fine grid, on the C2 surface (N = 24,576 coarse
    nodes, N_up = 393,216 fine nodes, 1.55e11 fine pairs); a step is sl_eval_upsampled.  The
    oracle's sandwich is checked on the 6 x 24 x 24 surface (every node)."""
    import numpy as np
    import torch
    import oracle
    from capsule_inputs import RBC, fine_pou, make_surface, sh_force
    from capsule_inputs import workloads as W
    p = W.c2()
    n = p.surface.n
    X, _, F = resident(dev, p.surface.X, p.surface.w, p.f)
    Wa = torch.as_tensor(p.surface.W, device=dev)
    psi = torch.as_tensor(fine_pou(n), device=dev)
    fine_pairs = float((16 * p.N) ** 2)
    res = {"workload": "rbc_6x64x64_sh8 upsampled 4x (N_up = 393,216), delta_u = delta* (C = 1)",
           "fine_pairs": fine_pairs}
    outs = {}
    for prec in ("fp64", "mixed"):
        U = torch.empty((3, p.N), dtype=torch.float64, device=dev)
        t = time_steps(lambda: ctx.single_layer_upsampled(X, Wa, F, n, psi, precision=prec, out=U), steps, warmup)
        outs[prec] = U.t().cpu().numpy()
        res[prec] = {"ms_per_step": round(t * 1e3, 3), "gpair_s": round(fine_pairs / t / 1e9, 1)}
        log(f"[bench] upsampled C2 {prec}: {t * 1e3:.2f} ms/step  {res[prec]['gpair_s']:.0f} Gpair/s "
            f"(fine pairs)")
    res["mixed_vs_fp64"] = rel_inf(outs["mixed"], outs["fp64"])
    # parity with the oracle at a size it finishes in seconds
    m = 24
    s = make_surface(RBC, m)
    f = sh_force(s.x0, 64)
    t0 = time.perf_counter()
    ref = oracle.single_layer_upsampled(s.X, s.W, f, m, fine_pou(m))
    tm = time.perf_counter() - t0
    Xs, _, Fs = resident(dev, s.X, s.w, f)
    Ws = torch.as_tensor(s.W, device=dev)
    ps = torch.as_tensor(fine_pou(m), device=dev)
    res["oracle_check"] = {"surface": "rbc_6x24x24 (N_up = 55,296)", "oracle_s": round(tm, 2)}
    for prec in ("fp64", "mixed"):
        u = ctx.single_layer_upsampled(Xs, Ws, Fs, m, ps, precision=prec)
        torch.cuda.synchronize()
        res["oracle_check"][f"eps_{prec}"] = rel_inf(u.cpu().numpy(), ref)
    log(f"[bench] upsampled: mixed vs fp64 {res['mixed_vs_fp64']:.2e}; vs oracle (6x24x24) fp64 "
        f"{res['oracle_check']['eps_fp64']:.2e}, mixed {res['oracle_check']['eps_mixed']:.2e}")
    return res


def fmm_leg(P, ctx, dev, log, steps=3, warmup=1):
    """The single-level FMM of Sec. 5 against the direct sum on the shape of the paper's FMM table
    (the a = 0.6 ellipsoid, reduced volume 0.9) at the upsampled sizes of its rows (m = 32, 64, 96:
    N_up = 6 (4 (m - 1))^2 = 92,256, 381,024 and 866,400 points), delta* per patch, SH density,
    k = 100 clusters and p = 5, 6, 8 points per cube edge (N_eq = 98, 152, 296 against the table's
    96, 128, 256).  A step is one evaluation: sl_eval (direct) or sl_eval_fmm (clustering, fit,
    near and far fields); eps_FMM is against the direct sum on the same GPU, in FP64."""
    import torch
    from capsule_inputs import ELLIPSOID_PAPER, make_surface, sh_force
    out = {"workload": "ellipsoid 0.6:1:1 at N_up of the paper's FMM table, delta* per patch, "
                       "SH density, k = 100", "rows": []}
    for m, p in ((32, 5), (64, 6), (96, 8)):
        n = 4 * (m - 1)
        t0 = time.perf_counter()
        s = make_surface(ELLIPSOID_PAPER, n)
        f = sh_force(s.x0, 9000 + m)
        X, w, F = resident(dev, s.X, s.w, f)
        D = ctx.patch_delta(X, n)
        torch.cuda.synchronize()
        row = {"m": m, "N_up": s.N, "p_edge": p, "N_eq": p ** 3 - (p - 2) ** 3}
        U = torch.empty((3, s.N), dtype=torch.float64, device=dev)
        V = torch.empty((3, s.N), dtype=torch.float64, device=dev)
        for prec in ("fp64", "mixed"):
            td = time_steps(lambda: ctx.single_layer(X, w, F, 0.0, delta_tgt=D, precision=prec, out=U),
                            steps, warmup)
            tf = time_steps(lambda: ctx.single_layer_fmm(X, w, F, 0.0, delta_tgt=D, k=100, p_edge=p,
                                                         precision=prec, out=V), steps, warmup)
            row[prec] = {"direct_ms": round(td * 1e3, 2), "fmm_ms": round(tf * 1e3, 2),
                         "speedup": round(td / tf, 3),
                         "eps_fmm_vs_direct": rel_inf(V.t().cpu().numpy(), U.t().cpu().numpy())}
            log(f"[bench] FMM m={m} N_up={s.N} p={p} {prec}: direct {td * 1e3:.1f} ms, FMM {tf * 1e3:.1f} ms "
                f"(x{td / tf:.2f}), eps_FMM {row[prec]['eps_fmm_vs_direct']:.1e}  "
                f"({time.perf_counter() - t0:.0f} s)")
        out["rows"].append(row)
        del X, w, F, D, U, V
    return out


def roofline(precision, pairs, near, kern_ms, workload):
    """Vector-ALU roofline of the pair kernel: algorithmic flops per launch (28 per far pair, 49
    per pair within the smoothing radius, exact counts) over its average launch duration, against
    the published vector peak of the precision it computes in.  `traffic` is the HBM bytes per
    launch from the stored rocprofv3 PMC runs of this workload, while they match the kernel's code."""
    flops = FLOPS_FAR * (pairs - near) + FLOPS_NEAR * near
    achieved = flops / (kern_ms * 1e-3) / 1e12
    peak = PEAK_TFLOPS[precision]
    traffic = None
    if os.path.exists(PMC_FILE):
        rec = json.load(open(PMC_FILE))
        entry = rec.get("workloads", {}).get(workload, {}).get(precision)
        if entry and rec.get("pair_kernel_sha") == pair_kernel_sha():
            traffic = entry["hbm_bytes_per_launch"]
    return {"bound": "alu", "achieved": round(achieved, 3), "peak": peak, "unit": "TFLOP/s",
            "frac": round(achieved / peak, 4), "traffic": traffic,
            "kernel_ms": round(kern_ms, 4), "flops_per_launch": flops,
            "flops_per_pair": {"far": FLOPS_FAR, "near": FLOPS_NEAR}, "near_pairs": near,
            "pairs": pairs, "algorithmic_bytes_per_launch": 24 * 2 * int(math.isqrt(pairs)) +
            (64 if precision == "fp64" else 96) * int(math.isqrt(pairs))}


def cpu_baseline(prob):
    """The oracle as it stands, on the host cores, over the whole workload (all targets).
    Returns the baseline record and the oracle's result (the reference for eps)."""
    import oracle
    oracle.build(force=False)
    threads = oracle.max_threads()
    t0 = time.perf_counter()
    ref = oracle.single_layer(prob.surface.X, prob.surface.w, prob.f, prob.delta)
    dt = time.perf_counter() - t0
    return ({"value": round(prob.N ** 2 / dt / 1e9, 4), "unit": "Gpair/s", "cores": threads,
             "kind": "oracle", "seconds": round(dt, 3),
             "sample": f"all {prob.N} targets x {prob.N} sources of the same surface and density"},
            ref)


def rel_inf(u, ref):
    import numpy as np
    return float(np.max(np.abs(u - ref)) / np.max(np.abs(ref)))


def pct(xs, q):
    import numpy as np
    return float(np.percentile(np.asarray(xs), q)) if len(xs) else None


def run_stream(ctx, P, handles, fs, us, pairs, arrivals, precision, spin):
    """Submit request k at arrivals[k] seconds after the start; poll until all are done.
    Returns (makespan s, latencies s = completion - scheduled arrival)."""
    n = len(handles)
    done_at = [None] * n
    rid_of = {}
    t0 = time.perf_counter()
    k = 0
    outstanding = []
    next_note = 20.0
    while k < n or outstanding:
        now = time.perf_counter() - t0
        if now > next_note:
            log(f"[bench] stream: {k} submitted, {n - k + len(outstanding) - (n - k)} outstanding "
                f"after {now:.0f} s")
            next_note += 20.0
        while k < n and arrivals[k] <= now:
            rid = ctx.submit_prepared(handles[k], fs[k], us[k], precision=precision)
            rid_of[rid] = k
            outstanding.append(rid)
            k += 1
        still = []
        for rid in outstanding:
            st, done = P.sl_poll(ctx.ptr, rid)
            P.check(st, "sl_poll")
            if done:
                done_at[rid_of[rid]] = time.perf_counter() - t0
            else:
                still.append(rid)
        outstanding = still
        if spin:
            time.sleep(spin)
    makespan = max(done_at)
    return makespan, [done_at[i] - arrivals[i] for i in range(n)]


def serving_leg(P, dev, log, check_oracle=True):
    """The request stream: 256 capsules (sphere / ellipsoid 1:0.8:0.5 / RBC, n log-uniform in
    [16, 192]), surfaces registered (resident) first; then a burst at t = 0 (capacity) and
    Poisson arrivals at 50% and 90% of the measured capacity, in mixed and in FP64, plus the
    same requests evaluated one at a time with sl_eval in FP64.  Every burst result is checked
    against the oracle on up to 256 sampled targets per request."""
    import numpy as np
    import torch
    from capsule_inputs import workloads as W
    t_gen = time.perf_counter()
    stream = W.serving_stream()
    probs = [r.problem() for r in stream.requests]
    log(f"[bench] serving stream: {len(probs)} requests generated in "
        f"{time.perf_counter() - t_gen:.1f} s")
    pairs = [p.N * p.N for p in probs]
    total = float(sum(pairs))
    out = {"workload": "256 requests: sphere / ellipsoid 1:0.8:0.5 / RBC, N = 6 n^2, n "
                       "log-uniform in [16, 192], SH density, delta = 2h",
           "total_pairs": total, "requests": len(probs)}
    refs = None
    if check_oracle:
        import oracle
        rng_t = np.random.default_rng(W.SEED_C4 + 2)
        t0 = time.perf_counter()
        refs = []
        for p in probs:
            idx = np.sort(rng_t.choice(p.N, size=min(256, p.N), replace=False))
            refs.append((idx, oracle.single_layer(p.surface.X, p.surface.w, p.f, p.delta,
                                                  targets=p.surface.X[idx])))
        log(f"[bench] serving: oracle on sampled targets in {time.perf_counter() - t0:.1f} s")
    with P.Context(0, hbm_budget_bytes=8 << 30) as ctx:
        t = lambda a: torch.as_tensor(a, device=dev)
        handles = [ctx.register_surface(t(p.surface.X), t(p.surface.w), p.delta) for p in probs]
        fs = [t(np.ascontiguousarray(p.f.T)) for p in probs]
        us = [torch.empty_like(f) for f in fs]
        torch.cuda.synchronize()
        rng = np.random.default_rng(W.SEED_C4 + 1)
        for prec in ("mixed", "fp64"):
            run_stream(ctx, P, handles[:8], fs[:8], us[:8], pairs[:8], [0.0] * 8, prec, 0)  # warm
            mk, lat = run_stream(ctx, P, handles, fs, us, pairs, [0.0] * len(probs), prec, 0)
            rec = {"burst": {"makespan_s": round(mk, 4), "gpair_s": round(total / mk / 1e9, 2),
                             "p50_ms": round(pct(lat, 50) * 1e3, 3),
                             "p99_ms": round(pct(lat, 99) * 1e3, 3)}}
            if refs is not None:
                eps = [rel_inf(u.t().cpu().numpy()[idx], ref) for u, (idx, ref) in zip(us, refs)]
                rec["burst"]["max_eps_vs_oracle"] = max(eps)
            cap_rps = len(probs) / mk
            for load in (0.5, 0.9):
                rate = load * cap_rps
                gaps = rng.exponential(1.0 / rate, size=len(probs))
                arrivals = list(np.cumsum(gaps) - gaps[0])
                mk2, lat2 = run_stream(ctx, P, handles, fs, us, pairs, arrivals, prec, 0)
                rec[f"poisson_{load}"] = {
                    "rate_hz": round(rate, 2), "offered_load": load,
                    "makespan_s": round(mk2, 4), "gpair_s": round(total / mk2 / 1e9, 2),
                    "p50_ms": round(pct(lat2, 50) * 1e3, 3), "p99_ms": round(pct(lat2, 99) * 1e3, 3),
                    "max_ms": round(max(lat2) * 1e3, 3)}
                log(f"[bench] serving {prec}: Poisson at {rate:.0f}/s (load {load}): "
                    f"p50 {pct(lat2, 50) * 1e3:.2f} ms p99 {pct(lat2, 99) * 1e3:.2f} ms")
            out[prec] = rec
            log(f"[bench] serving {prec}: burst {total / mk / 1e9:.0f} Gpair/s"
                + (f", max eps {rec['burst']['max_eps_vs_oracle']:.2e}" if refs is not None else ""))
        st = ctx.stats()
        out["kernel_launches"] = int(st.kernel_launches)
        out["requests_done"] = int(st.requests_done)
        # one at a time, FP64, sl_eval on the same GPU
        ev = P.Context(0)
        Xs = [t(p.surface.X) for p in probs]
        ws = [t(p.surface.w) for p in probs]
        Fs = [t(p.f) for p in probs]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for p, X, w, F in zip(probs, Xs, ws, Fs):
            ev.single_layer(X, w, F, p.delta, precision="fp64")
            torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        ev.close()
        out["fp64_one_at_a_time"] = {"seconds": round(dt, 4), "gpair_s": round(total / dt / 1e9, 2)}
    return out


def memory_leg(P, dev, log, n_large=2, n_small=62, passes=2, budgets=("full", "one_large")):
    """The memory-admitted stream: n_large capsules of N = 6 * 512^2 interleaved with n_small ones
    (n log-uniform in [16, 64]), RBC and ellipsoid, evaluated in `passes` passes with a fresh
    density each time (the stated size is 64 + 2,000; the default run is a scaled sample).  The
    client keeps surfaces resident across passes (least recently used first out): when a
    registration is refused for lack of memory it releases idle surfaces, else retires its oldest
    request first.  Run with the full budget (everything stays resident) and with a budget that
    holds one large capsule but not two (the large surfaces are evicted and registered again).
    Surfaces and SH bases are generated once per (shape, n) and densities when submitted."""
    import collections
    import numpy as np
    import torch
    from capsule_inputs import forces as FO
    from capsule_inputs import make_surface
    from capsule_inputs import workloads as W
    stream = W.memory_admitted_stream(n_large=n_large, n_small=n_small)
    t0 = time.perf_counter()
    surfs, bases = {}, {}
    for r in stream.requests:
        if (r.shape, r.n) not in surfs:
            surfs[(r.shape, r.n)] = make_surface(W.SERVING_SHAPES[r.shape], r.n)
        if r.n not in bases:
            bases[r.n] = FO.real_sph_harm_all(surfs[(r.shape, r.n)].x0)
    log(f"[bench] memory stream: {len(stream.requests)} capsules, {len(surfs)} surfaces generated in "
        f"{time.perf_counter() - t0:.1f} s")

    class Req:
        def __init__(self, i, r):
            self.surface = surfs[(r.shape, r.n)]
            self.N = r.N
            self.delta = W.delta_2h(r.n)
            self.seed, self.i, self.n = r.seed, i, r.n

        def density(self, k):
            seed = self.seed if k == 0 else W.SEED_C5 * 100 + 7 * k + self.i
            return bases[self.n] @ FO.sh_coefficients(seed).T

    probs = [Req(i, r) for i, r in enumerate(stream.requests)]
    total = float(sum(p.N * p.N for p in probs)) * passes
    n_big = max(p.N for p in probs)
    per_point = 85                       # resident surface (49 B) + mixed staging (36 B) per point
    all_budgets = {"full": 16 << 30, "one_large": int(1.15 * per_point * n_big)}
    budgets = {k: all_budgets[k] for k in budgets}
    out = {"workload": f"{n_large} capsules N = {n_big} + {n_small} with n in [16, 64] (RBC / "
                       f"ellipsoid), SH density, delta = 2h, {passes} pass(es) with fresh densities; "
                       "surfaces kept resident, least recently used released when memory is short",
           "total_pairs": total, "requests": len(probs) * passes}
    for bname, budget in budgets.items():
        for prec in ("mixed", "fp64"):
            with P.Context(0, hbm_budget_bytes=budget) as ctx:
                torch.cuda.synchronize()
                cur = torch.cuda.current_stream()
                resident = collections.OrderedDict()      # capsule -> handle, LRU order
                inflight = collections.deque()            # (rid, capsule, keep-alive)
                busy = collections.Counter()
                registrations = evictions = 0
                peak = 0

                def retire_done():
                    while inflight and ctx.poll(inflight[0][0]):
                        busy[inflight.popleft()[1]] -= 1

                def make_room(nbytes, keep):
                    """Release idle surfaces (least recently used first), then retire the
                    oldest requests, until nbytes more fit the budget."""
                    nonlocal evictions
                    while budget - int(ctx.stats().bytes_admitted) < nbytes:
                        idle = [c for c in resident if busy[c] == 0 and c != keep]
                        if idle:
                            ctx.release_surface(resident.pop(idle[0]))
                            evictions += 1
                        elif inflight:
                            rid0, c0, _ = inflight.popleft()
                            ctx.wait(rid0, 120.0)
                            busy[c0] -= 1
                        else:
                            return

                t0 = time.perf_counter()
                next_note = 20.0
                for k in range(passes):
                    for i, p in enumerate(probs):
                        if time.perf_counter() - t0 > next_note:
                            log(f"[bench] memory stream {bname} {prec}: pass {k}, capsule {i} of "
                                f"{len(probs)} after {next_note:.0f} s")
                            next_note += 20.0
                        np_i = -(-p.N // 256) * 256   # padded nodes: 49 B each resident
                        if i in resident:
                            resident.move_to_end(i)
                        else:
                            X = torch.as_tensor(p.surface.X, device=dev)
                            w = torch.as_tensor(p.surface.w, device=dev)
                            cur.synchronize()    # this stream only: the serving kernel keeps running
                            make_room(49 * np_i, None)
                            while True:
                                try:
                                    resident[i] = ctx.register_surface(X, w, p.delta)
                                    registrations += 1
                                    break
                                except P.SlError as e:
                                    if e.status != P.SL_EBUSY or not (resident or inflight):
                                        raise
                                    make_room(budget, None)   # everything idle goes
                        make_room(ctx.request_bytes(resident[i], prec), i)
                        f = torch.as_tensor(np.ascontiguousarray(p.density(k).T), device=dev)
                        u = torch.empty_like(f)
                        cur.synchronize()
                        rid = ctx.submit_prepared(resident[i], f, u, precision=prec)
                        inflight.append((rid, i, (f, u)))
                        busy[i] += 1
                        peak = max(peak, int(ctx.stats().bytes_admitted))
                        retire_done()
                while inflight:
                    rid0, c0, _ = inflight.popleft()
                    ctx.wait(rid0, 120.0)
                    if time.perf_counter() - t0 > next_note:
                        log(f"[bench] memory stream {bname} {prec}: draining, {len(inflight)} in "
                            f"flight after {next_note:.0f} s")
                        next_note += 20.0
                dt = time.perf_counter() - t0
            out[f"{bname}_{prec}"] = {"budget_bytes": budget, "seconds": round(dt, 3),
                                      "gpair_s": round(total / dt / 1e9, 2),
                                      "registrations": registrations, "evictions": evictions,
                                      "peak_bytes_admitted": peak}
            log(f"[bench] memory stream {bname} {prec}: {dt:.2f} s  {total / dt / 1e9:.0f} Gpair/s  "
                f"registrations {registrations} evictions {evictions}  peak {peak / 2**30:.2f} GiB")
    return out


def secondary_c2(P, ctx, dev, steps, warmup, with_oracle):
    """The 6 x 64 x 64 surface (N = 24,576): both precisions, roofline of the pair kernel (its
    average duration from the library's events in a second pass), error against the oracle over
    every target."""
    from capsule_inputs import workloads as W
    prob = W.c2()
    tens = resident(dev, prob.surface.X, prob.surface.w, prob.f)
    pairs = prob.N * prob.N
    near = count_near(tens[0], prob.delta, [RHO_EXACT64, 5.0])
    out = {"workload": "rbc_6x64x64_sh8", "N": prob.N, "delta": prob.delta}
    outs = {}
    for prec in ("fp64", "mixed"):
        ms, kern_ms, outs[prec] = measure_precision(ctx, P, prob, tens, prec, steps, warmup)
        near_p = near[RHO_EXACT64] if prec == "fp64" else near[5.0]
        out[prec] = {"ms_per_step": round(ms, 4), "gpair_s": round(pairs / (ms * 1e-3) / 1e9, 3),
                     "roofline": roofline(prec, pairs, near_p, kern_ms, "rbc_6x64x64_sh8")}
        log(f"[bench] C2 {prec}: {ms:.3f} ms/step  {out[prec]['gpair_s']:.1f} Gpair/s  pair kernel "
            f"{kern_ms:.3f} ms  {out[prec]['roofline']['frac'] * 100:.1f}% of peak")
    if with_oracle:
        rec, ref = cpu_baseline(prob)
        out["oracle"] = rec
        for prec in ("fp64", "mixed"):
            out[prec]["eps_vs_oracle"] = rel_inf(outs[prec].t().cpu().numpy(), ref)
            log(f"[bench] C2 {prec}: eps vs oracle (all targets) {out[prec]['eps_vs_oracle']:.2e}")
    return out, prob, tens


def write_pmc(prefix: str) -> None:
    """profiles/pmc_pair_kernel.json from the FETCH_SIZE and WRITE_SIZE passes of both workloads
    (rocprofv3 --pmc <counter> --output-format csv -d <prefix>_<c3|c2>_<counter> -o run -- python3
    bench.py --workload <c3|c2> ... --copy-bytes 1073741824): per-dispatch means of each kernel,
    scaled to bytes by what the same counter read for the device copy of known size.  Host only."""
    import csv
    import re

    def load(path):
        d = {}
        for r in csv.DictReader(open(path)):
            key = re.sub(r"\(.*", "", r["Kernel_Name"].replace("void ", "")
                         .replace("sl::(anonymous namespace)::", ""))
            d.setdefault(key, []).append(float(r["Counter_Value"]))
        return d

    rec = {"pair_kernel_sha": pair_kernel_sha(), "copy_bytes": COPY_BYTES_PMC, "workloads": {}}
    for tag, wl in (("c3", "rbc_6x256x256_sh8"), ("c2", "rbc_6x64x64_sh8")):
        F = load(f"{prefix}_{tag}_FETCH_SIZE/run_counter_collection.csv")
        W = load(f"{prefix}_{tag}_WRITE_SIZE/run_counter_collection.csv")
        # the calibration copy is the largest copy dispatch (the runtime's small copies are KiB)
        copy = [k for k in F if "copyBuffer" in k]
        if len(copy) != 1:
            raise SystemExit(f"{prefix}_{tag}: no calibration copy")
        cf, cw = max(F[copy[0]]), max(W[copy[0]])
        fs, ws = COPY_BYTES_PMC / (cf * 1024), COPY_BYTES_PMC / (cw * 1024)
        out = {"copy_fetch_kib": cf, "copy_write_kib": cw, "fetch_scale": round(fs, 4),
               "write_scale": round(ws, 4)}
        for k in sorted(F):
            if not (k.startswith("k_pair<") or k == "k_reduce"):
                continue
            f, w = sum(F[k]) / len(F[k]), sum(W[k]) / len(W[k])
            fb, wb = round(f * 1024 * fs), round(w * 1024 * ws)
            if k == "k_reduce":
                out[k] = {"fetch_bytes": fb, "write_bytes": wb}
                continue
            prec = "mixed" if k.split("<")[1].split(",")[2].strip() == "true" else "fp64"
            out[prec] = {"kernel": k, "dispatches": len(F[k]), "fetch_kib": round(f, 1),
                         "write_kib": round(w, 1), "fetch_bytes": fb, "write_bytes": wb,
                         "hbm_bytes_per_launch": fb + wb}
        rec["workloads"][wl] = out
    with open(PMC_FILE, "w") as fh:
        json.dump(rec, fh, indent=1)
        fh.write("\n")
    print(json.dumps(rec, indent=1))


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=30)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--precision", choices=["mixed", "fp64"], default="mixed")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true",
                    help="only the headline workload (no C2, per-patch delta, upsampling, serving)")
    ap.add_argument("--no-serving", action="store_true", help="skip the serving leg")
    ap.add_argument("--no-memory-stream", action="store_true",
                    help="skip the memory-admitted stream leg")
    ap.add_argument("--c5-full", action="store_true",
                    help="run the memory-admitted stream at its stated size (64 capsules of "
                         "N = 1,572,864 and 2,000 small ones, three passes, with the full budget "
                         "and with one that holds a single large capsule; about 20 minutes)")
    ap.add_argument("--workload", choices=["c3", "c2"], default="c3",
                    help="workload of the timed step: RBC 6x256x256 (the headline) or RBC 6x64x64 "
                         "(for counter runs of the smaller case)")
    ap.add_argument("--copy-bytes", type=int, default=0,
                    help="also run one device copy of this many bytes (PMC calibration)")
    ap.add_argument("--write-pmc", metavar="PREFIX",
                    help="write the stored HBM traffic from the csv output of the FETCH_SIZE and "
                         "WRITE_SIZE passes under PREFIX_<c3|c2>_<counter>/ and exit (no GPU)")
    args = ap.parse_args()
    if args.write_pmc:
        write_pmc(args.write_pmc)
        return
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
    rho64 = P.sl_get_param(ctx.ptr, P.SL_PARAM_RHO64)
    wl, tag, prob, seed = (("rbc_6x256x256_sh8", "C3", W.c3(), W.SEED_C3) if args.workload == "c3"
                           else ("rbc_6x64x64_sh8", "C2", W.c2(), W.SEED_C2))
    tens = resident(dev, prob.surface.X, prob.surface.w, prob.f)
    pairs = prob.N * prob.N
    log(f"[bench] workload {wl}: N={prob.N}, delta={prob.delta:.6g}")
    t0 = time.perf_counter()
    near = count_near(tens[0], prob.delta, [RHO_EXACT64, 5.0])
    log(f"[bench] exact near-pair counts in {time.perf_counter() - t0:.1f} s: "
        f"r < 6.9 delta {near[RHO_EXACT64]}, r < 5 delta {near[5.0]}")

    res = {}
    outs = {}
    for prec in ("fp64", "mixed"):
        ms, kern_ms, launches, med, outs[prec] = measure_headline(ctx, P, prob, tens, prec,
                                                                  args.steps, args.warmup)
        near_p = near[RHO_EXACT64] if prec == "fp64" else near[5.0]
        res[prec] = {"ms_per_step": round(ms, 4), "gpair_s": round(pairs / (ms * 1e-3) / 1e9, 3),
                     "median_ms_30_reps": round(med, 4), "timed_pair_launches": launches,
                     "roofline": roofline(prec, pairs, near_p, kern_ms, wl)}
        log(f"[bench] {tag} {prec}: {ms:.3f} ms/step (median {med:.3f})  {res[prec]['gpair_s']:.1f} "
            f"Gpair/s  pair kernel {kern_ms:.3f} ms  {res[prec]['roofline']['frac'] * 100:.1f}% of peak")

    head = res[args.precision]
    other = "fp64" if args.precision == "mixed" else "mixed"
    line = {
        "metric": "Gpair/s regularized Stokeslet sum, FP32-mixed vs FP64; p50/p99 latency",
        "value": head["gpair_s"], "unit": "Gpair/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": head["ms_per_step"], "higher_is_better": True,
        "scaling": "strong", "vs_baseline": None,
        "dtype": "f32+f64" if args.precision == "mixed" else "f64",
        "data": "synthetic",
        "config": {"workload": wl, "N": prob.N, "delta": prob.delta, "mu": 1.0,
                   "precision": args.precision, "rho64": rho64, "seed": seed,
                   "step": "sl_eval: sort + pack + pair kernel + reduction, all N targets"},
        "roofline": {k: head["roofline"][k] for k in
                     ("bound", "achieved", "peak", "unit", "frac", "traffic")},
        "roofline_detail": head["roofline"],
        "median_ms_30_reps": head["median_ms_30_reps"],
        other: res[other],
    }

    if not args.no_cpu_baseline:
        log("[bench] cpu baseline: oracle on the host (4,096 sampled targets; 512 on one core)")
        idx = W.c3_subset(prob.N, 4096)
        line["cpu_baseline"], ref = cpu_baseline_sampled(prob, idx, idx[:512])
        log(f"[bench] oracle: {line['cpu_baseline']['value']:.3f} Gpair/s on "
            f"{line['cpu_baseline']['cores']} threads, {line['cpu_baseline']['one_core']['value']:.4f} "
            f"on one ({line['cpu_baseline']['cpu_model']})")
        for prec in ("fp64", "mixed"):
            e = rel_inf(outs[prec].t().cpu().numpy()[idx], ref)
            (line if prec == args.precision else line[prec])["eps_vs_oracle_4096_targets"] = e
            log(f"[bench] {tag} {prec}: eps vs oracle (4,096 targets) {e:.2e}")
    del outs

    if not args.no_extras:
        line["c2"], p2, t2 = secondary_c2(P, ctx, dev, 100, 5, not args.no_cpu_baseline)
        line["patch_delta"] = patch_delta_leg(P, ctx, p2, t2, log)
        line["upsampled"] = upsample_leg(P, ctx, dev, log)
        del t2
        line["fmm"] = fmm_leg(P, ctx, dev, log)
        if not args.no_serving:
            line["serving"] = serving_leg(P, dev, log)
            line["p50_ms"] = line["serving"]["mixed"]["poisson_0.9"]["p50_ms"]
            line["p99_ms"] = line["serving"]["mixed"]["poisson_0.9"]["p99_ms"]
        if not args.no_memory_stream:
            line["memory_stream_sample"] = memory_leg(P, dev, log)
    if args.c5_full:
        line["memory_stream_full"] = memory_leg(P, dev, log, n_large=64, n_small=2000, passes=3,
                                                budgets=("full", "one_large"))

    if args.copy_bytes:
        a = torch.empty(args.copy_bytes // 8, dtype=torch.float64, device=dev).fill_(1.0)
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        line["copy_calibration_bytes"] = args.copy_bytes

    ctx.close()
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
