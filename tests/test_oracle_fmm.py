"""Pins of the oracle's single-level FMM (oracle/fmm.py, Sec. 5) against what the mathematics
fixes, independently of its own code path:

* the clustering is a fixed point of Lloyd's iteration (every point at its nearest centroid by an
  independently computed distance; every centroid the mean of its points within the quantization);
* the equivalent sources of the unit box reproduce, outside the far cube, the plain-Stokeslet field
  of sources inside the box (uniqueness of the exterior Stokes solution), with an error that falls
  with the grid;
* with a single cluster every target's sources are near and the FMM is the plain sum;
* every far pair is outside the source cluster's check surface and at least 6.9 delta apart (so
  the plain kernel equals the regularized one there);
* the error against the direct sum falls with the equivalent grid, within the bounds of the decades
  the paper's FMM table reports (6E-3, 4E-5, 5E-6 for N_eq = 96, 128, 256).
"""
import math

import numpy as np
import pytest

from capsule_inputs import ELLIPSOID_PAPER, RBC, SPHERE, make_surface, sh_force


def test_kmeans_is_a_lloyd_fixed_point():
    from oracle import fmm
    s = make_surface(RBC, 20)
    lab, C, it = fmm.kmeans(s.X, 50)
    assert it < fmm.KMEANS_MAX_ITER
    # nearest centroid, distances by numpy's norm (a different formula): ties allowed
    D = np.linalg.norm(s.X[:, None, :] - C[None, :, :], axis=2)
    assert np.all(D[np.arange(s.N), lab] <= D.min(axis=1) * (1 + 1e-12))
    # centroids = means of their points to the quantization step
    ext = float((s.X.max(0) - s.X.min(0)).max())
    step = 2.0 ** (math.frexp(ext)[1] - 24)
    for j in range(50):
        P = s.X[lab == j]
        if len(P):
            assert np.all(np.abs(P.mean(axis=0) - C[j]) <= step)
    # deterministic
    lab2, C2, _ = fmm.kmeans(s.X, 50)
    assert np.array_equal(lab, lab2) and np.array_equal(C, C2)


@pytest.mark.parametrize("p,bound", [(4, 5e-2), (6, 3e-4), (8, 3e-5)])
def test_equivalent_sources_reproduce_the_exterior_field(p, bound):
    """Random Stokeslets inside the unit box, targets on cubes of half width 3 to 6 around it: the
    equivalent sources fitted on the check surface give the same velocity to the bound."""
    from oracle import fmm
    import oracle
    rng = np.random.default_rng(p)
    src = rng.uniform(-1, 1, (300, 3))
    g = rng.standard_normal((300, 3))
    t = rng.uniform(-1, 1, (400, 3))
    t = t / np.abs(t).max(axis=1, keepdims=True) * rng.uniform(3.0, 6.0, (400, 1))
    E = fmm.cube_points(p)
    assert E.shape[0] == p ** 3 - (p - 2) ** 3
    v = oracle.stokeslet(src, g, fmm.ALPHA_CHECK * E)
    phi = fmm.unit_operator(p) @ np.concatenate([v[:, 0], v[:, 1], v[:, 2]])
    ne = E.shape[0]
    eq = np.stack([phi[:ne], phi[ne:2 * ne], phi[2 * ne:]], axis=1)
    far = oracle.stokeslet(fmm.ALPHA_EQ * E, eq, t)
    exact = oracle.stokeslet(src, g, t)
    assert np.abs(far - exact).max() / np.abs(exact).max() < bound


def test_single_cluster_is_the_plain_sum():
    import oracle
    from oracle import fmm
    s = make_surface(SPHERE, 8)
    f = sh_force(s.x0, 8)
    d = 2 * math.pi / 9
    u = fmm.single_layer_fmm(s.X, s.w, f, d, k=1, p=4)
    ref = oracle.single_layer(s.X, s.w, f, d)
    assert np.abs(u - ref).max() / np.abs(ref).max() < 1e-14


def test_far_pairs_are_outside_the_check_surface_and_the_smoothing():
    import oracle
    from oracle import fmm
    n = 40
    s = make_surface(ELLIPSOID_PAPER, n)
    f = sh_force(s.x0, 3)
    dt = oracle.patch_delta(s.X, n)
    _, d = fmm.single_layer_fmm(s.X, s.w, f, 0.0, delta_tgt=dt, k=100, p=4, details=True)
    lab, o, a, near = d["labels"], d["centre"], d["half_width"], d["near"]
    n_far = 0
    for T in range(100):
        PT = s.X[lab == T]
        for S in range(100):
            if near[T, S] or not len(PT) or not np.any(lab == S):
                continue
            n_far += 1
            assert np.all(np.abs(PT - o[S]).max(axis=1) > fmm.ALPHA_CHECK * a[S])
            PS = s.X[lab == S]
            r = np.linalg.norm(PT[:, None, :] - PS[None, :, :], axis=2)
            assert r.min() >= fmm.RHO_EXACT * dt[lab == T].max()
    assert n_far > 1000


@pytest.mark.slow
def test_error_against_direct_falls_with_the_grid():
    """The paper's a = 0.6 ellipsoid, delta* per patch, k = 100: eps_FMM against the direct sum
    at p = 4, 6, 8 (N_eq = 56, 152, 296) falls by orders of magnitude, below the decades of the
    paper's FMM table."""
    import oracle
    from oracle import fmm
    n = 48
    s = make_surface(ELLIPSOID_PAPER, n)
    f = sh_force(s.x0, 7)
    dt = oracle.patch_delta(s.X, n)
    ref = oracle.single_layer(s.X, s.w, f, 0.0, delta_tgt=dt)
    errs = []
    for p in (4, 6, 8):
        u = fmm.single_layer_fmm(s.X, s.w, f, 0.0, delta_tgt=dt, k=100, p=p)
        errs.append(np.abs(u - ref).max() / np.abs(ref).max())
    assert errs[0] > 10 * errs[1] and errs[1] > 5 * errs[2], errs
    assert errs[0] < 6e-3 and errs[1] < 4e-5 and errs[2] < 5e-6, errs
