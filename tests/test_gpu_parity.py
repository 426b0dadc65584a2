"""Parity of the HIP path (through the C ABI) with the CPU FP64 oracle.

Tolerances are the relative infinity-norm error eps = ||u - u_ref||_inf / ||u_ref||_inf of
Sec. 4.1: 1e-12 for SL_FP64 and 1e-6 for SL_MIXED.
"""
import math

import numpy as np
import pytest

from capsule_inputs import ELLIPSOID_SERVING, RBC, SPHERE, Shape, make_surface, sh_force
from capsule_inputs import workloads as W

pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-12, "mixed": 1e-6}


@pytest.fixture(scope="module")
def ctx():
    import torch
    import paper_2310_13908_amd as P
    assert torch.cuda.is_available()
    c = P.Context(0)
    yield c
    c.close()


def gpu_eval(ctx, X, w, f, delta, mu=1.0, targets=None, delta_tgt=None, precision="fp64"):
    import torch
    dev = torch.device("cuda", 0)
    t = lambda a: None if a is None else torch.as_tensor(np.asarray(a, dtype=np.float64), device=dev)
    u = ctx.single_layer(t(X), t(w), t(f), delta, mu=mu, targets=t(targets),
                         delta_tgt=t(delta_tgt), precision=precision)
    torch.cuda.synchronize()
    return u.cpu().numpy()


def eps(u, ref):
    return float(np.max(np.abs(u - ref)) / np.max(np.abs(ref)))


@pytest.fixture(scope="module")
def c2_ref():
    import oracle
    p = W.c2()
    return p, oracle.single_layer(p.surface.X, p.surface.w, p.f, p.delta)


# ----------------------------------------------------------------------------------------------
@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_c1_sphere(ctx, precision):
    """Unit sphere, 6 x 18 x 18 nodes, uniform traction: oracle parity and the 2/3 e_z answer."""
    import oracle
    p = W.c1()
    u = gpu_eval(ctx, p.surface.X, p.surface.w, p.f, p.delta, precision=precision)
    ref = oracle.single_layer(p.surface.X, p.surface.w, p.f, p.delta)
    assert eps(u, ref) < TOL[precision]
    assert eps(u, np.tile([0, 0, 2 / 3], (p.N, 1))) < 2e-4


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("n", [1, 2, 5, 11, 21, 40])
def test_small_surfaces_ragged(ctx, n, precision):
    """Sizes from a single cluster to several tiles with a ragged tail (N = 6 n^2)."""
    import oracle
    s = make_surface(RBC, n)
    f = sh_force(s.x0, 100 + n)
    d = 2 * math.pi / (n + 1)
    u = gpu_eval(ctx, s.X, s.w, f, d, mu=0.7, precision=precision)
    ref = oracle.single_layer(s.X, s.w, f, d, mu=0.7)
    assert eps(u, ref) < TOL[precision]


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_c2_rbc_full(ctx, c2_ref, precision):
    """Biconcave surface, 6 x 64 x 64 nodes, SH density: every target against the oracle."""
    p, ref = c2_ref
    u = gpu_eval(ctx, p.surface.X, p.surface.w, p.f, p.delta, precision=precision)
    assert eps(u, ref) < TOL[precision]


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_c3_rbc_sampled(ctx, precision):
    """6 x 256 x 256 nodes (N = 393,216), the launch configuration the benchmark times; the
    workload's 4,096 sampled targets recomputed by the oracle over all sources."""
    import oracle
    p = W.c3()
    u = gpu_eval(ctx, p.surface.X, p.surface.w, p.f, p.delta, precision=precision)
    idx = W.c3_subset(p.N, 4096)
    ref = oracle.single_layer(p.surface.X, p.surface.w, p.f, p.delta, targets=p.surface.X[idx])
    assert eps(u[idx], ref) < TOL[precision]
    assert np.all(np.isfinite(u))


@pytest.mark.parametrize("n", [104, 105])
def test_sort_paths_at_the_scan_threshold(ctx, n):
    """N = 6 n^2 on either side of 2^16 = 64 sort blocks of 1024 keys (64,896 and 66,150 points):
    below it two radix passes whose scatters take their offsets from the raw counts, above it
    three passes with the three-kernel scan of the counts.  Targets = sources and distinct
    targets (a second sort with the same scratch, two passes after three for n = 105), 256 sampled
    targets each against the oracle."""
    import oracle
    s = make_surface(RBC, n)
    f = sh_force(s.x0, 300 + n)
    d = 2 * math.pi / (n + 1)
    idx = np.sort(np.random.default_rng(n).choice(s.N, size=256, replace=False))
    for precision in ("fp64", "mixed"):
        u = gpu_eval(ctx, s.X, s.w, f, d, precision=precision)
        ref = oracle.single_layer(s.X, s.w, f, d, targets=s.X[idx])
        assert eps(u[idx], ref) < TOL[precision]
        T = s.X[idx] * 1.001
        u = gpu_eval(ctx, s.X, s.w, f, d, targets=T, precision=precision)
        assert eps(u, oracle.single_layer(s.X, s.w, f, d, targets=T)) < TOL[precision]


@pytest.mark.parametrize("n_t", [65536, 65537])
@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_sort_few_sources_many_targets(ctx, precision, n_t):
    """4,704 sources (a two-pass sort) and 2^16 or 2^16 + 1 distinct targets in one call: the
    last size sorted in two passes (64 blocks of 1024 keys, offsets from the raw counts) and the
    first in three (65 blocks, the three-kernel count scan), each sort reusing the scratch of
    the sources' sort.  Every target against the oracle."""
    import oracle
    s = make_surface(RBC, 28)
    f = sh_force(s.x0, 41)
    d = 2 * math.pi / 29
    rng = np.random.default_rng(41)
    T = s.X[rng.integers(0, s.N, n_t)] + rng.normal(scale=0.05, size=(n_t, 3))
    u = gpu_eval(ctx, s.X, s.w, f, d, targets=T, precision=precision)
    ref = oracle.single_layer(s.X, s.w, f, d, targets=T)
    assert eps(u, ref) < TOL[precision]


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_distinct_targets(ctx, precision):
    """Targets off the nodes: on-surface nodes, points near and far from the surface, and points
    that coincide exactly with sources (r = 0 handled by the limit)."""
    import oracle
    s = make_surface(ELLIPSOID_SERVING, 9)
    f = sh_force(s.x0, 5)
    rng = np.random.default_rng(9)
    T = np.concatenate([s.X[::7], s.X[:40] * 1.02, rng.standard_normal((200, 3)) * 2.0,
                        s.X[100:103]])
    d = 2 * math.pi / 10
    u = gpu_eval(ctx, s.X, s.w, f, d, targets=T, precision=precision)
    ref = oracle.single_layer(s.X, s.w, f, d, targets=T)
    assert eps(u, ref) < TOL[precision]


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_per_target_delta(ctx, precision):
    import oracle
    s = make_surface(RBC, 14)
    f = sh_force(s.x0, 6)
    d0 = 2 * math.pi / 15
    dt = d0 * (0.5 + np.random.default_rng(2).random(s.N))
    u = gpu_eval(ctx, s.X, s.w, f, 0.0, delta_tgt=dt, precision=precision)
    ref = oracle.single_layer(s.X, s.w, f, 0.0, delta_tgt=dt)
    assert eps(u, ref) < TOL[precision]
    # distinct targets with per-target delta
    T = s.X[::3] + 0.01
    dtt = dt[::3]
    u = gpu_eval(ctx, s.X, s.w, f, 0.0, targets=T, delta_tgt=dtt, precision=precision)
    ref = oracle.single_layer(s.X, s.w, f, 0.0, targets=T, delta_tgt=dtt)
    assert eps(u, ref) < TOL[precision]


@pytest.mark.parametrize("precision,rho64", [("fp64", 0.0), ("mixed", 0.0), ("mixed", 1.0)])
def test_per_target_delta_above_2_17_targets(ctx, precision, rho64):
    """RBC 6 x 160 x 160 (N = 153,600 > 2^17 targets, where the FP64 path keeps two targets per
    lane) with the paper's per-patch delta = delta* (eq. (regparam)) and with a random per-target
    delta; 256 sampled targets against the oracle over all sources.  Mixed without and with the
    FP64 zone."""
    import oracle
    n = 160
    s = make_surface(RBC, n)
    f = sh_force(s.x0, 160)
    idx = np.sort(np.random.default_rng(160).choice(s.N, size=256, replace=False))
    dstar = oracle.patch_delta(s.X, n)
    drand = (2 * math.pi / (n + 1)) * (0.5 + np.random.default_rng(161).random(s.N))
    ctx.set_rho64(rho64)
    try:
        for dt in (dstar, drand):
            u = gpu_eval(ctx, s.X, s.w, f, 0.0, delta_tgt=dt, precision=precision)
            ref = oracle.single_layer(s.X, s.w, f, 0.0, targets=s.X[idx], delta_tgt=dt[idx])
            assert eps(u[idx], ref) < TOL[precision]
            assert np.all(np.isfinite(u))
    finally:
        ctx.set_rho64(0.0)


@pytest.mark.parametrize("precision,rho64,per_target", [("fp64", 0.0, False), ("fp64", 0.0, True),
                                                        ("mixed", 0.0, False), ("mixed", 1.0, False)])
def test_smoothing_profile_single_source(ctx, precision, rho64, per_target):
    """One source, targets at r/delta from 0 (coincident) through the exact-smoothing cut (6.9)
    to 9, in many directions: every target's velocity is a single pair term, so this checks the
    device s1/r and s2/r^3 per target, not in a norm.  The points include both sides of every
    boundary of the double-precision table's rows (q = (r/delta)^2 = 1 and 2^e (1 + j/4)) and of
    its end at q = 48, past which its identity row applies.  FP64 runs with one delta and with the
    same delta given per target (the per-target-delta kernel); mixed without a double-precision
    zone (the default) and with rho64 = 1."""
    import oracle
    rng = np.random.default_rng(17)
    delta = 0.037
    edges = np.array([1.0] + [2.0 ** e * (1 + j / 4) for e in range(6) for j in range(4)] + [48.0])
    rho_edges = np.sqrt(np.concatenate([edges * (1 - 1e-13), edges, edges * (1 + 1e-13)]))
    rho = np.concatenate([[0.0, 1e-12, 1e-8, 1e-5, 1e-3, 0.1, 0.4999, 0.5, 0.5001],
                          np.linspace(0.0, 9.0, 1801)[1:], [4.9999, 5.0, 5.0001, 6.8999, 6.9, 6.9001],
                          rho_edges])
    dirs = rng.standard_normal((rho.size, 3))
    dirs /= np.linalg.norm(dirs, axis=1, keepdims=True)
    src = np.array([[0.31, -0.72, 0.18]])
    T = src + rho[:, None] * delta * dirs
    g = np.array([[0.8, -1.3, 0.45]])
    ctx.set_rho64(rho64)
    try:
        if per_target:
            u = gpu_eval(ctx, src, [0.02], g, 0.0, targets=T, delta_tgt=np.full(rho.size, delta),
                         precision=precision)
        else:
            u = gpu_eval(ctx, src, [0.02], g, delta, targets=T, precision=precision)
    finally:
        ctx.set_rho64(0.0)
    ref = oracle.single_layer(src, [0.02], g, delta, targets=T)
    rel = np.linalg.norm(u - ref, axis=1) / np.linalg.norm(ref, axis=1)
    # FP64: double precision everywhere.  Mixed: double precision below r/delta = rho64, single
    # precision (smoothed below 5) elsewhere -- a per-pair bound there, not the norm bound.
    if precision == "fp64":
        tol = np.full(rho.shape, 2e-14)
    else:
        tol = np.where(rho < 0.99 * rho64, 2e-14, 3e-6)
    assert np.all(rel <= tol), (rho[rel > tol][:5], rel[rel > tol][:5])


def test_degenerate_sizes(ctx):
    import torch
    import oracle
    import paper_2310_13908_amd as P
    dev = torch.device("cuda", 0)
    # single source = single target: only the self term
    x = np.array([[0.3, -0.2, 0.9]])
    f = np.array([[1.0, 2.0, -0.5]])
    u = gpu_eval(ctx, x, [0.25], f, 0.2, mu=1.5)
    assert eps(u, oracle.single_layer(x, [0.25], f, 0.2, mu=1.5)) < 1e-15
    # exactly duplicated nodes (two sources at one point)
    X = np.array([[0.0, 0.0, 1.0], [0.0, 0.0, 1.0], [0.5, 0.1, 0.2]])
    F = np.array([[1.0, 0.0, 0.0], [0.0, 1.0, 0.0], [0.0, 0.0, 1.0]])
    for prec in ("fp64", "mixed"):
        u = gpu_eval(ctx, X, [0.1, 0.2, 0.3], F, 0.3, precision=prec)
        assert eps(u, oracle.single_layer(X, [0.1, 0.2, 0.3], F, 0.3)) < TOL[prec]
    # no sources: zeros; no targets: nothing enqueued
    T = torch.ones((5, 3), dtype=torch.float64, device=dev)
    U = torch.full((3, 5), 7.0, dtype=torch.float64, device=dev)
    e = torch.empty(0, dtype=torch.float64, device=dev)
    st = P.sl_eval(ctx.ptr, P.SL_FP64, 0, e.data_ptr(), e.data_ptr(), e.data_ptr(), e.data_ptr(),
                   e.data_ptr(), e.data_ptr(), e.data_ptr(), 5, T[:, 0].contiguous().data_ptr(),
                   T[:, 1].contiguous().data_ptr(), T[:, 2].contiguous().data_ptr(), 0.1, None, 1.0,
                   U[0].data_ptr(), U[1].data_ptr(), U[2].data_ptr(), 0)
    assert st == P.SL_OK
    torch.cuda.synchronize()
    assert torch.all(U == 0)
    st = P.sl_eval(ctx.ptr, P.SL_FP64, 0, None, None, None, None, None, None, None, 0, None, None,
                   None, 0.1, None, 1.0, None, None, None, 0)
    assert st == P.SL_OK


def test_deterministic_and_translation_rotation(ctx):
    """Bit-identical repeats; results covariant under rigid motions (compared to the oracle on
    the moved inputs, and to the rotated unmoved result)."""
    import oracle
    s = make_surface(RBC, 30)
    f = sh_force(s.x0, 8)
    d = 2 * math.pi / 31
    for prec in ("fp64", "mixed"):
        u1 = gpu_eval(ctx, s.X, s.w, f, d, precision=prec)
        u2 = gpu_eval(ctx, s.X, s.w, f, d, precision=prec)
        assert np.array_equal(u1, u2)
        shift = np.array([100.0, -50.0, 20.0])
        ut = gpu_eval(ctx, s.X + shift, s.w, f, d, precision=prec)
        assert eps(ut, oracle.single_layer(s.X + shift, s.w, f, d)) < TOL[prec]
        th = 0.9
        R = np.array([[math.cos(th), -math.sin(th), 0], [math.sin(th), math.cos(th), 0], [0, 0, 1]])
        ur = gpu_eval(ctx, s.X @ R.T, s.w, f @ R.T, d, precision=prec)
        assert eps(ur, u1 @ R.T) < 10 * TOL[prec]


def test_reciprocity_and_linearity(ctx):
    s = make_surface(SPHERE, 24)
    f, g = sh_force(s.x0, 31), sh_force(s.x0, 32)
    d = 2 * math.pi / 25
    uf = gpu_eval(ctx, s.X, s.w, f, d)
    ug = gpu_eval(ctx, s.X, s.w, g, d)
    a, b = np.sum(s.w[:, None] * g * uf), np.sum(s.w[:, None] * f * ug)
    assert abs(a - b) <= 1e-12 * (abs(a) + abs(b))
    u3 = gpu_eval(ctx, s.X, s.w, 2 * f - g, d, mu=0.25)
    assert eps(u3, 4 * (2 * uf - ug)) < 1e-13


def test_invalid_arguments(ctx):
    import torch
    import paper_2310_13908_amd as P
    dev = torch.device("cuda", 0)
    X = torch.rand((3, 100), dtype=torch.float64, device=dev)
    U = torch.empty((3, 100), dtype=torch.float64, device=dev)
    p = [X[0].data_ptr(), X[1].data_ptr(), X[2].data_ptr()]
    wv = torch.ones(100, dtype=torch.float64, device=dev).data_ptr()

    def call(delta=0.1, mu=1.0, n=100, out=None, prec=P.SL_FP64):
        o = out or [U[0].data_ptr(), U[1].data_ptr(), U[2].data_ptr()]
        return P.sl_eval(ctx.ptr, prec, n, *p, wv, *p, n, None, None, None, delta, None, mu, *o, 0)

    assert call() == P.SL_OK
    for bad in (0.0, -1.0, float("nan"), float("inf")):
        assert call(delta=bad) == P.SL_EINVAL
        assert call(mu=bad) == P.SL_EINVAL
    assert call(n=-1) == P.SL_EINVAL
    assert call(prec=7) == P.SL_EINVAL
    assert call(out=[U[0].data_ptr(), U[0].data_ptr(), U[2].data_ptr()]) == P.SL_EINVAL   # overlap
    assert call(out=[X[0].data_ptr(), U[1].data_ptr(), U[2].data_ptr()]) == P.SL_EINVAL   # aliases input
    assert "alias" in P.sl_last_error()
    torch.cuda.synchronize()


def test_rho64_parameter(ctx, c2_ref):
    """A larger double-precision zone in the mixed path moves the result towards FP64; the
    default is no zone."""
    p, ref = c2_ref
    import paper_2310_13908_amd as P
    assert P.sl_set_param(ctx.ptr, P.SL_PARAM_RHO64, -0.1) == P.SL_EINVAL
    assert P.sl_set_param(ctx.ptr, P.SL_PARAM_RHO64, float("nan")) == P.SL_EINVAL
    assert P.sl_get_param(ctx.ptr, P.SL_PARAM_RHO64) == 0.0
    errs = {}
    try:
        for rho64 in (0.0, 0.5, 1.0, 5.0, 12.0):
            ctx.set_rho64(rho64)
            errs[rho64] = eps(gpu_eval(ctx, p.surface.X, p.surface.w, p.f, p.delta,
                                       precision="mixed"), ref)
    finally:
        ctx.set_rho64(0.0)
    assert all(e < TOL["mixed"] for e in errs.values()), errs
    assert errs[12.0] < errs[0.0] and errs[12.0] < errs[1.0]


@pytest.mark.parametrize("precision,rho64", [("fp64", 0.0), ("mixed", 0.0), ("mixed", 1.0)])
def test_launch_shapes(precision, rho64):
    """Every targets-per-lane and work granularity gives the same sums to the tolerance, with one
    delta and with a per-target delta, in FP64 and in mixed without and with the FP64 zone.  N =
    6 * 21^2 = 2646 pads to 2816 = 11 blocks of 256: with 4 targets per lane the last workgroup
    of four blocks is short, and distinct targets (1000 points) pad to a different count."""
    import oracle
    import paper_2310_13908_amd as P
    s = make_surface(RBC, 21)
    f = sh_force(s.x0, 77)
    d = 2 * math.pi / 22
    T = s.X[::3] * 1.01
    dt = d * (0.6 + 0.8 * np.random.default_rng(21).random(s.N))
    dtt = dt[::3]
    ref = oracle.single_layer(s.X, s.w, f, d)
    ref_t = oracle.single_layer(s.X, s.w, f, d, targets=T)
    ref_v = oracle.single_layer(s.X, s.w, f, 0.0, delta_tgt=dt)
    ref_vt = oracle.single_layer(s.X, s.w, f, 0.0, targets=T, delta_tgt=dtt)
    with P.Context(0) as c:
        c.set_rho64(rho64)
        for R in (1, 2, 4):
            for wps in (1, 3, 16, 64, 256):
                P.check(P.sl_set_param(c.ptr, P.SL_PARAM_TARGETS_PER_LANE, float(R)))
                P.check(P.sl_set_param(c.ptr, P.SL_PARAM_WAVES_PER_SIMD, float(wps)))
                u = gpu_eval(c, s.X, s.w, f, d, precision=precision)
                assert eps(u, ref) < TOL[precision], (R, wps)
                u = gpu_eval(c, s.X, s.w, f, d, targets=T, precision=precision)
                assert eps(u, ref_t) < TOL[precision], (R, wps)
                u = gpu_eval(c, s.X, s.w, f, 0.0, delta_tgt=dt, precision=precision)
                assert eps(u, ref_v) < TOL[precision], (R, wps, "delta_tgt")
                u = gpu_eval(c, s.X, s.w, f, 0.0, targets=T, delta_tgt=dtt, precision=precision)
                assert eps(u, ref_vt) < TOL[precision], (R, wps, "delta_tgt, targets")


@pytest.fixture(scope="module")
def c5_large():
    """One capsule of the memory-admitted stream at its full size: ellipsoid 1:0.8:0.5,
    6 x 512 x 512 nodes (N = 1,572,864), SH density, delta = 2h; 64 sampled targets."""
    import oracle
    p = W.shape_sh(ELLIPSOID_SERVING, 512, W.SEED_C5)
    idx = np.sort(np.random.default_rng(W.SEED_C5).choice(p.N, size=64, replace=False))
    ref = oracle.single_layer(p.surface.X, p.surface.w, p.f, p.delta, targets=p.surface.X[idx])
    return p, idx, ref


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_largest_capsule_one_shot_and_served(ctx, c5_large, precision):
    """The largest surface of the workloads through sl_eval and through the serving path, on
    sampled targets recomputed by the oracle over all 1.57 M sources."""
    import torch
    p, idx, ref = c5_large
    u = gpu_eval(ctx, p.surface.X, p.surface.w, p.f, p.delta, precision=precision)
    assert eps(u[idx], ref) < TOL[precision]
    assert np.all(np.isfinite(u))
    dev = torch.device("cuda", 0)
    t = lambda a: torch.as_tensor(np.asarray(a, dtype=np.float64), device=dev)
    h = ctx.register_surface(t(p.surface.X), t(p.surface.w), p.delta)
    rid, _ = ctx.submit(h, t(p.f), precision=precision)
    us = ctx.wait(rid, 120.0).cpu().numpy()
    ctx.release_surface(h)
    assert eps(us[idx], ref) < TOL[precision]
