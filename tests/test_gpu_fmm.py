"""The single-level FMM of Sec. 5 through the C ABI (sl_eval_fmm): the clustering bit for bit and
the result element by element against the oracle's FMM (oracle/fmm.py), the limit in which every
cluster is near (the plain sum), and the error against the direct sum falling with the number of
equivalent points."""
import math

import numpy as np
import pytest

from capsule_inputs import ELLIPSOID_PAPER, RBC, SPHERE, make_surface, sh_force

pytestmark = pytest.mark.gpu

# FP64: the single-layer bar.  The device and the oracle fit the equivalent densities with two
# different least-squares solvers (Householder QR of the stacked Tikhonov system on the host against
# LAPACK's SVD-based solver); the two operators differ by up to ~6e-10 of their largest entry, but
# only in directions that the Tikhonov weight and the far field damp: u differs by at most 4e-13 on
# the cases below.  Mixed: the single-precision bar of the plain sum.
TOL = {"fp64": 1e-12, "mixed": 1e-6}


def eps(u, ref):
    return float(np.max(np.abs(u - ref)) / np.max(np.abs(ref)))


@pytest.fixture(scope="module")
def ctx():
    import torch
    import paper_2310_13908_amd as P
    assert torch.cuda.is_available()
    c = P.Context(0)
    yield c
    c.close()


def dev(a):
    import torch
    return torch.as_tensor(np.asarray(a, dtype=np.float64), device=torch.device("cuda", 0))


def run_fmm(ctx, s, f, delta, dt, k, p, precision, max_iter=100):
    import torch
    u, lab = ctx.single_layer_fmm(dev(s.X), dev(s.w), dev(f), delta,
                                  delta_tgt=None if dt is None else dev(dt), k=k, p_edge=p,
                                  max_iter=max_iter, precision=precision, labels=True)
    torch.cuda.synchronize()
    return u.cpu().numpy(), lab.cpu().numpy()


CASES = [  # shape, n, per-patch delta, k, p
    (ELLIPSOID_PAPER, 24, True, 100, 4),
    (ELLIPSOID_PAPER, 48, True, 100, 6),
    (RBC, 40, False, 100, 5),
    (SPHERE, 10, False, 37, 4),
]


@pytest.fixture(scope="module")
def oracle_fmm():
    import oracle
    from oracle import fmm
    out = {}
    for shape, n, pd, k, p in CASES:
        s = make_surface(shape, n)
        f = sh_force(s.x0, 900 + n)
        dt = oracle.patch_delta(s.X, n) if pd else None
        delta = 0.0 if pd else 2 * math.pi / (n + 1)
        u, d = fmm.single_layer_fmm(s.X, s.w, f, delta, delta_tgt=dt, k=k, p=p, details=True)
        out[(shape.kind, n)] = (s, f, delta, dt, k, p, u, d)
    return out


@pytest.mark.parametrize("case", [(c[0].kind, c[1]) for c in CASES])
@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_fmm_matches_the_oracle(ctx, oracle_fmm, case, precision):
    s, f, delta, dt, k, p, ref, d = oracle_fmm[case]
    print(f"[fmm] {case} {precision} N={s.N} k={k} p={p}", flush=True)
    u, lab = run_fmm(ctx, s, f, delta, dt, k, p, precision)
    assert np.array_equal(lab, d["labels"])
    e = eps(u, ref)
    print(f"[fmm] eps vs oracle FMM {e:.3e}", flush=True)
    assert e < TOL[precision], e


@pytest.fixture(scope="module")
def large_case():
    """The a = 0.6 ellipsoid with 6 x 160 x 160 = 153,600 points (delta* per patch, k = 100,
    p = 5): the oracle's FMM on the targets of three clusters only."""
    import oracle
    from oracle import fmm
    n = 160
    s = make_surface(ELLIPSOID_PAPER, n)
    f = sh_force(s.x0, n)
    dt = oracle.patch_delta(s.X, n)
    ref, d = fmm.single_layer_fmm(s.X, s.w, f, 0.0, delta_tgt=dt, k=100, p=5, details=True,
                                  only=(0, 41, 99))
    return s, f, dt, ref, d


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_fmm_above_2_17_targets(ctx, large_case, precision):
    """Above 2^17 targets, where the FP64 pair kernels keep two targets per lane: clusters bit for
    bit, u on three clusters' targets element by element."""
    s, f, dt, ref, d = large_case
    u, lab = run_fmm(ctx, s, f, 0.0, dt, 100, 5, precision)
    assert np.array_equal(lab, d["labels"])
    sel = np.isin(lab, (0, 41, 99))
    e = eps(u[sel], ref[sel])
    print(f"[fmm] N={s.N} {precision} eps vs oracle FMM on {sel.sum()} targets {e:.3e}", flush=True)
    assert e < TOL[precision], e


def test_single_cluster_is_the_plain_sum(ctx):
    """k = 1: every target's only cluster is near, so the FMM is the direct sum."""
    import torch
    s = make_surface(RBC, 12)
    f = sh_force(s.x0, 12)
    d = 2 * math.pi / 13
    u, lab = run_fmm(ctx, s, f, d, None, 1, 4, "fp64")
    ref = ctx.single_layer(dev(s.X), dev(s.w), dev(f), d).cpu().numpy()
    torch.cuda.synchronize()
    assert np.all(lab == 0)
    assert eps(u, ref) < 1e-13


def test_error_against_direct_falls_with_the_equivalent_grid(ctx):
    """On the paper's a = 0.6 ellipsoid with delta* per patch: the FMM's error against the direct
    sum (sl_eval) falls with the points per cube edge."""
    import oracle
    n = 48
    s = make_surface(ELLIPSOID_PAPER, n)
    f = sh_force(s.x0, 48)
    dt = oracle.patch_delta(s.X, n)
    direct = ctx.single_layer(dev(s.X), dev(s.w), dev(f), 0.0, delta_tgt=dev(dt)).cpu().numpy()
    errs = []
    for p in (4, 6, 8):
        u, _ = run_fmm(ctx, s, f, 0.0, dt, 100, p, "fp64")
        errs.append(eps(u, direct))
    print(f"[fmm] eps vs direct p=4,6,8: {errs}", flush=True)
    assert errs[0] > errs[1] > errs[2]
    assert errs[0] < 1e-3 and errs[2] < 1e-6


def test_invalid_arguments(ctx):
    import paper_2310_13908_amd as P
    s = make_surface(RBC, 4)
    f = sh_force(s.x0, 4)
    for kw in ({"k": 0}, {"k": s.N + 1}, {"p": 2}, {"p": 13}, {"max_iter": 0}):
        args = dict(k=10, p=4, max_iter=100)
        args.update(kw)
        with pytest.raises(P.SlError) as e:
            run_fmm(ctx, s, f, 0.3, None, args["k"], args["p"], "fp64", args["max_iter"])
        assert e.value.status == P.SL_EINVAL
