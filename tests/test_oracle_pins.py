"""Pins for the CPU FP64 oracle: it is checked against what the paper and the mathematics
fix, never against itself.  A dropped term, a wrong sign, a swapped index or a wrong weight
in the oracle fails at least one of these."""
import math
import os

import mpmath
import numpy as np
import pytest
from scipy import integrate

from capsule_inputs import ELLIPSOID_PAPER, RBC, SPHERE, make_surface, sh_force
from capsule_inputs import workloads as W

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
SQPI = math.sqrt(math.pi)


def stokeslet(d, f, mu=1.0):
    """Textbook free-space Stokeslet velocity of a point force f at offset d."""
    r = np.linalg.norm(d)
    return (f / r + np.dot(f, d) * d / r ** 3) / (8 * math.pi * mu)


# ---------------------------------------------------------------------------------------------
# Kernel factors s1, s2 (Sec. 3.4)
# ---------------------------------------------------------------------------------------------
def test_kernel_limits_printed_in_paper(oracle_lib):
    """Sec. 3.4: s1(r/d)/r -> 16/(3 d sqrt(pi)), s2(r/d)/r^3 -> 32/(3 d^3 sqrt(pi))."""
    lim = {}
    for line in open(os.path.join(GOLDEN, "kernel_limits.txt")):
        if line.strip() and not line.startswith("#"):
            name, num, den, pw = line.split()
            lim[name] = (float(num), float(den), int(pw))
    for d in (0.05, 0.33, 1.7):
        K1_0 = lim["K1"][0] / (lim["K1"][1] * d ** lim["K1"][2] * SQPI)
        K2_0 = lim["K2"][0] / (lim["K2"][1] * d ** lim["K2"][2] * SQPI)
        K1, K2 = oracle_lib.kernel(0.0, d)
        assert K1 == pytest.approx(K1_0, rel=1e-15)
        # the printed formula, evaluated at small rho, approaches the printed limits
        for rho in (1e-2, 3e-3):
            K1, K2 = oracle_lib.kernel(rho * d, d)
            assert abs(K1 / K1_0 - 1) < 2 * rho ** 2
            assert abs(K2 / K2_0 - 1) < 2 * rho ** 2


@pytest.mark.parametrize("which", [0, 1])
def test_smoothing_moments(oracle_lib, which):
    """The O(delta^5) accuracy claimed in Sec. 3.4 rests on int_0^inf rho^k (s - 1) drho = 0 for
    k = 0, 2; the k = 4 moments are -16/(15 sqrt(pi)) (s1) and -32/(5 sqrt(pi)) (s2), closed forms
    from the erfc and Gaussian moments.  Any altered coefficient in s1 or s2 breaks one of them."""
    def g(p, k):
        return p ** k * (oracle_lib.smoothing(p)[which] - 1.0)
    m = [integrate.quad(g, 0, 12, args=(k,), epsabs=1e-14, epsrel=1e-13, limit=200)[0]
         for k in (0, 2, 4)]
    assert abs(m[0]) < 1e-13 and abs(m[1]) < 1e-13
    expect4 = -16 / (15 * SQPI) if which == 0 else -32 / (5 * SQPI)
    assert m[2] == pytest.approx(expect4, rel=1e-12)


def test_smoothing_tends_to_one(oracle_lib):
    """Far from the target the regularized kernel is the plain Stokeslet (s1 = s2 = 1)."""
    for p in (7.0, 9.0, 20.0):
        s1, s2 = oracle_lib.smoothing(p)
        assert s1 == 1.0 and s2 == 1.0


def test_far_pair_is_the_textbook_stokeslet(oracle_lib):
    rng = np.random.default_rng(3)
    xs = rng.standard_normal((1, 3))
    f = rng.standard_normal((1, 3))
    t = xs + np.array([[2.0, -1.0, 0.5]])
    for delta in (0.01, 0.1):
        u = oracle_lib.single_layer(xs, [0.7], f, delta, mu=1.3, targets=t)[0]
        ref = 0.7 * stokeslet(t[0] - xs[0], f[0], mu=1.3)
        assert np.allclose(u, ref, rtol=1e-14, atol=0)


def test_self_pair_uses_the_limit(oracle_lib):
    """A target on its own source: u = w f * 16/(3 delta sqrt(pi)) / (8 pi mu)."""
    x = np.array([[0.2, -0.4, 1.1]])
    f = np.array([[1.0, -2.0, 0.5]])
    u = oracle_lib.single_layer(x, [0.3], f, 0.25, mu=2.0)[0]
    assert np.allclose(u, 0.3 * f[0] * 16 / (3 * 0.25 * SQPI) / (16 * math.pi), rtol=1e-15)


# ---------------------------------------------------------------------------------------------
# Closed forms on the sphere
# ---------------------------------------------------------------------------------------------
def test_sphere_uniform_traction_drag():
    """Rigid sphere: uniform traction f gives u = 2 a f / (3 mu) on the surface (Stokes drag).
    The configuration of the first workload (n = 18) and its h-refinement."""
    import oracle
    for n, tol in [(18, 2e-4), (31, 1e-5), (47, 1e-6)]:
        p = W.sphere_uniform(n)
        u = oracle.single_layer(p.surface.X, p.surface.w, p.f, p.delta)
        assert oracle.rel_inf_error(u, np.tile([0, 0, 2 / 3], (p.N, 1))) < tol


def test_sphere_radius_and_viscosity_scaling():
    import oracle
    a, mu = 1.7, 0.4
    s = make_surface(type(SPHERE)("sphere", (a, a, a)), 31)
    f = np.tile([0.3, -1.0, 0.2], (s.N, 1))
    u = oracle.single_layer(s.X, s.w, f, 2 * a * math.pi / 32, mu=mu)
    assert oracle.rel_inf_error(u, np.tile(2 * a * f[0] / (3 * mu), (s.N, 1))) < 2e-5


def test_sphere_rigid_rotation():
    """Traction (3 mu / a) Omega x x on a sphere gives u = Omega x x (torque 8 pi mu a^3 Omega)."""
    import oracle
    Om = np.array([0.3, -0.5, 0.8])
    for n, tol in [(31, 2e-5), (63, 3e-7)]:
        s = make_surface(SPHERE, n)
        u = oracle.single_layer(s.X, s.w, 3.0 * np.cross(Om, s.X), 2 * math.pi / (n + 1))
        assert oracle.rel_inf_error(u, np.cross(Om, s.X)) < tol


def test_single_layer_of_normal_vanishes_with_stated_order():
    """S[n] = 0 on a closed surface (divergence-free Stokeslet).  With delta = 2h the regularized
    sum converges to 0 at the O(delta^5) order stated in Sec. 3.4 on the paper's a = 0.6
    ellipsoid: the observed slope rises to ~5 under h-refinement."""
    import oracle
    errs = []
    ns = [31, 63, 127, 255]
    for n in ns:
        s = make_surface(ELLIPSOID_PAPER, n)
        d = 2 * math.pi / (n + 1)
        idx = np.random.default_rng(1).choice(s.N, size=min(s.N, 400), replace=False)
        u = oracle.single_layer(s.X, s.w, s.normal, d, targets=s.X[idx])
        ref = oracle.single_layer(s.X, s.w, np.tile([0, 0, 1.0], (s.N, 1)), d, targets=s.X[idx])
        errs.append(np.abs(u).max() / np.abs(ref).max())
    slopes = [math.log2(errs[i] / errs[i + 1]) for i in range(len(ns) - 1)]
    assert errs[-1] < 1e-7
    assert slopes[0] < slopes[1] < slopes[2]
    assert 4.5 < slopes[-1] < 5.5


# ---------------------------------------------------------------------------------------------
# Exact discrete structure
# ---------------------------------------------------------------------------------------------
@pytest.fixture(scope="module")
def small_rbc():
    s = make_surface(RBC, 12)
    return s, sh_force(s.x0, 11), sh_force(s.x0, 12), 2 * math.pi / 13


def test_reciprocity(small_rbc):
    """The kernel is a symmetric tensor even in d, so sum_i w_i f'_i . u[f]_i is symmetric in
    (f, f').  Catches a target weight in place of a source weight and a transposed kernel."""
    import oracle
    s, f, g, d = small_rbc
    uf = oracle.single_layer(s.X, s.w, f, d)
    ug = oracle.single_layer(s.X, s.w, g, d)
    a = np.sum(s.w[:, None] * g * uf)
    b = np.sum(s.w[:, None] * f * ug)
    assert abs(a - b) <= 1e-13 * (abs(a) + abs(b))


def test_linearity_and_viscosity(small_rbc):
    import oracle
    s, f, g, d = small_rbc
    u = oracle.single_layer(s.X, s.w, 2.0 * f - 3.0 * g, d, mu=0.5)
    ref = 2 * (2.0 * oracle.single_layer(s.X, s.w, f, d) - 3.0 * oracle.single_layer(s.X, s.w, g, d))
    assert oracle.rel_inf_error(u, ref) < 1e-14


def test_translation_and_rotation(small_rbc):
    import oracle
    s, f, _, d = small_rbc
    u = oracle.single_layer(s.X, s.w, f, d)
    ut = oracle.single_layer(s.X + np.array([5.0, -3.0, 2.0]), s.w, f, d)
    assert oracle.rel_inf_error(ut, u) < 1e-13
    th = 0.7
    R = np.array([[1, 0, 0], [0, math.cos(th), -math.sin(th)], [0, math.sin(th), math.cos(th)]])
    R = R @ np.array([[math.cos(1.1), 0, math.sin(1.1)], [0, 1, 0], [-math.sin(1.1), 0, math.cos(1.1)]])
    ur = oracle.single_layer(s.X @ R.T, s.w, f @ R.T, d)
    assert oracle.rel_inf_error(ur, u @ R.T) < 1e-13


def test_per_target_delta(small_rbc):
    """delta_tgt[i] applies to target i only: each row equals a scalar-delta call."""
    import oracle
    s, f, _, d = small_rbc
    dt = d * (0.5 + np.random.default_rng(5).random(s.N))
    u = oracle.single_layer(s.X, s.w, f, 0.0, delta_tgt=dt)
    for i in (0, 17, s.N - 1):
        ui = oracle.single_layer(s.X, s.w, f, dt[i], targets=s.X[i:i + 1])[0]
        assert np.array_equal(u[i], ui)
    assert np.array_equal(oracle.single_layer(s.X, s.w, f, 0.0, delta_tgt=np.full(s.N, d)),
                          oracle.single_layer(s.X, s.w, f, d))


def test_rejects_bad_arguments(small_rbc):
    import oracle
    s, f, _, d = small_rbc
    for bad in (0.0, -1.0, float("nan"), float("inf")):
        with pytest.raises(ValueError):
            oracle.single_layer(s.X, s.w, f, bad)
        with pytest.raises(ValueError):
            oracle.single_layer(s.X, s.w, f, d, mu=bad)


# ---------------------------------------------------------------------------------------------
# Brute force at 40 digits on a tiny surface
# ---------------------------------------------------------------------------------------------
def _brute_force_mp(X, w, f, delta, mu):
    mpmath.mp.dps = 40
    sq = mpmath.sqrt(mpmath.pi)
    dl = mpmath.mpf(delta)
    N = X.shape[0]
    Xm = [[mpmath.mpf(float(v)) for v in row] for row in X]
    fm = [[mpmath.mpf(float(v)) for v in row] for row in f]
    wm = [mpmath.mpf(float(v)) for v in w]
    out = np.zeros((N, 3))
    for i in range(N):
        acc = [mpmath.mpf(0)] * 3
        for j in range(N):
            d = [Xm[i][k] - Xm[j][k] for k in range(3)]
            r = mpmath.sqrt(d[0] ** 2 + d[1] ** 2 + d[2] ** 2)
            if r == 0:
                a, b = 16 / (3 * dl * sq), mpmath.mpf(0)
            else:
                p = r / dl
                e = mpmath.exp(-p * p) / sq
                a = (mpmath.erf(p) - mpmath.mpf(2) / 3 * p * (2 * p ** 2 - 5) * e) / r
                b = (mpmath.erf(p) - mpmath.mpf(2) / 3 * p * (4 * p ** 4 - 14 * p ** 2 + 3) * e) / r ** 3
            fd = sum(fm[j][k] * d[k] for k in range(3))
            for k in range(3):
                acc[k] += wm[j] * (a * fm[j][k] + b * fd * d[k])
        for k in range(3):
            out[i, k] = float(acc[k] / (8 * mpmath.pi * mu))
    return out


def test_brute_force_40_digits():
    import oracle
    s = make_surface(RBC, 4)                   # N = 96
    f = sh_force(s.x0, 21)
    d = 2 * math.pi / 5
    ref = _brute_force_mp(s.X, s.w, f, d, 1.3)
    u = oracle.single_layer(s.X, s.w, f, d, mu=1.3)
    assert oracle.rel_inf_error(u, ref) < 5e-15


# ---------------------------------------------------------------------------------------------
# Per-patch regularization parameter delta = C delta* (Sec. 3.4, eq. (regparam))
# ---------------------------------------------------------------------------------------------
def planar_patch(n, fx, fy):
    """Nodes (fx(l), fy(l'), 0) of one n x n patch, (l, l') row-major."""
    l, lp = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    return np.stack([fx(l).ravel(), fy(lp).ravel(), np.zeros(n * n)], axis=1).astype(np.float64)


def test_patch_delta_uniform_grid_is_the_diagonal():
    """On a flat grid of spacings sx, sy the largest neighbour distance is the diagonal
    sqrt(sx^2 + sy^2); every node of the patch gets C times it."""
    import oracle
    for n, sx, sy, C in ((2, 1.0, 1.0, 1.0), (5, 0.3, 0.4, 1.0), (7, 0.02, 0.05, 2.5)):
        X = planar_patch(n, lambda l: sx * l, lambda lp: sy * lp)
        d = oracle.patch_delta(X, n, C=C)
        assert np.allclose(d, C * math.hypot(sx, sy), rtol=1e-15, atol=0)


def test_patch_delta_stretched_grid():
    """x = l^2, y = l': the widest cell is the last one, whose diagonal is sqrt((2n-3)^2 + 1)."""
    import oracle
    for n in (3, 6, 11):
        X = planar_patch(n, lambda l: l.astype(np.float64) ** 2, lambda lp: lp.astype(np.float64))
        assert np.allclose(oracle.patch_delta(X, n), math.hypot(2 * n - 3, 1.0), rtol=1e-15)


def test_patch_delta_single_node_has_no_neighbours():
    import oracle
    assert np.all(oracle.patch_delta(np.array([[0.1, 0.2, 0.3]] * 6), 1) == 0.0)


def test_patch_delta_per_patch_and_invariances():
    """Each patch gets its own delta*; delta* scales with the surface and is invariant under a
    rigid motion; on the 6-patch discretization it matches a brute force over all node pairs
    of a patch that are adjacent in the grid."""
    import oracle
    n = 9
    s = make_surface(RBC, n)
    d = oracle.patch_delta(s.X, n)
    per = d.reshape(6, n * n)
    assert np.all(per == per[:, :1])                     # constant on each patch
    l, lp = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    L, LP = l.ravel(), lp.ravel()
    adj = (np.abs(L[:, None] - L[None]) <= 1) & (np.abs(LP[:, None] - LP[None]) <= 1)
    for i in range(6):
        P = s.X[i * n * n:(i + 1) * n * n]
        dist = np.linalg.norm(P[:, None] - P[None], axis=-1)
        assert per[i, 0] == pytest.approx(dist[adj].max(), rel=1e-15)
    assert len(set(np.round(per[:, 0], 12))) > 1       # the RBC patches differ
    assert np.allclose(oracle.patch_delta(3.0 * s.X, n), 3.0 * d, rtol=1e-14)
    Q, _ = np.linalg.qr(np.random.default_rng(5).standard_normal((3, 3)))
    assert np.allclose(oracle.patch_delta(s.X @ Q.T + [1.0, -2.0, 0.5], n), d, rtol=1e-13)


def test_patch_delta_rejects_bad_arguments():
    import oracle
    with pytest.raises(ValueError):
        oracle.patch_delta(np.zeros((10, 3)), 3)          # not whole patches
    with pytest.raises(ValueError):
        oracle.patch_delta(np.zeros((9, 3)), 3, C=0.0)


# ---------------------------------------------------------------------------------------------
# Upsampling sandwich (Sec. 3.4, "Upsampling"): I_u, W_u, w_u, I_d
# ---------------------------------------------------------------------------------------------
def test_spline_resample_reproduces_bicubics():
    """Not-a-knot cubic splines reproduce every polynomial of degree <= 3 in each variable, and
    its u- and v-derivatives; an asymmetric one catches swapped axes or patch order."""
    import oracle
    from capsule_inputs import fine_grid
    n = 7
    tc, tf = fine_grid(n)
    P = lambda u, v, k: (1 + k) * (0.3 + u - 0.7 * u ** 3) * (2.0 - 0.4 * v ** 2 + 0.1 * v ** 3) + k * u * v
    Pu = lambda u, v, k: (1 + k) * (1 - 2.1 * u ** 2) * (2.0 - 0.4 * v ** 2 + 0.1 * v ** 3) + k * v
    Pv = lambda u, v, k: (1 + k) * (0.3 + u - 0.7 * u ** 3) * (-0.8 * v + 0.3 * v ** 2) + k * u
    Uc, Vc = np.meshgrid(tc, tc, indexing="ij")
    Uf, Vf = np.meshgrid(tf, tf, indexing="ij")
    F = np.concatenate([P(Uc, Vc, k).ravel() for k in range(6)])
    for du, dv, ref in ((0, 0, P), (1, 0, Pu), (0, 1, Pv)):
        G = oracle.spline_resample(F, n, tc, tf, du=du, dv=dv)
        want = np.concatenate([ref(Uf, Vf, k).ravel() for k in range(6)])
        assert np.allclose(G, want, rtol=0, atol=1e-11)


def test_fine_weights_upsample_the_area_element():
    """Sec. 3.6 (upsampling step): W_u = I_u W with the same spline operator as X and F, and the
    fine weights are psi_u W_u h_u^2 (eq. (smoothint) on the fine grid).  A coarse area element
    that is a bicubic in (u, v) on each patch is reproduced exactly by the not-a-knot splines, so
    the fine weights must equal psi_u times that bicubic at the fine nodes times h_u^2: a weight
    computed from anything else (the spline surface's own |X_u x X_v|, a coarse h, a missing
    psi_u) fails.  Factors 2 and 4."""
    import oracle
    from capsule_inputs import fine_grid, fine_pou
    n = 9
    s = make_surface(RBC, n)
    P = lambda u, v, k: (2.0 + 0.1 * k) + 0.3 * u - 0.05 * u ** 3 + 0.2 * v ** 2 * (1 + 0.1 * u) \
        - 0.01 * k * v ** 3
    for factor in (2, 4):
        tc, tf = fine_grid(n, factor)
        Uc, Vc = np.meshgrid(tc, tc, indexing="ij")
        Uf, Vf = np.meshgrid(tf, tf, indexing="ij")
        Wc = np.concatenate([P(Uc, Vc, k).ravel() for k in range(6)])
        Wf = np.concatenate([P(Uf, Vf, k).ravel() for k in range(6)])
        hf = math.pi / (factor * n + 1)
        psi = fine_pou(n, factor)
        Xu, wu = oracle.upsampled_surface(s.X, Wc, n, psi, factor)
        assert Xu.shape == (6 * (factor * n) ** 2, 3)
        assert np.allclose(wu, psi * Wf * hf * hf, rtol=1e-12, atol=0)


def test_upsampled_surface_converges_at_fourth_order():
    """I_u X against the exact positions of the fine nodes: O(h^4) (ratio ~16 per halving of h).
    The fine weights psi_u (I_u W) h_u^2 integrate the biconcave surface's area (1-D quadrature
    of the surface of revolution) with the fourth-order error of the spline interpolation of W:
    an error ratio near 16 per halving, and below 1e-5 at n = 24 and 1e-6 at n = 48.  Weights
    from the derivatives of the spline surface instead of I_u W miss these bounds (8.5e-5 at
    n = 24)."""
    import oracle
    from capsule_inputs import fine_pou, fine_positions
    from test_inputs import rbc_area_volume
    errs = []
    for n in (8, 16, 32):
        s = make_surface(SPHERE, n)
        Xu, wu = oracle.upsampled_surface(s.X, s.W, n, fine_pou(n))
        errs.append(np.abs(Xu - fine_positions(SPHERE, n)).max())
    assert errs[0] / errs[1] > 10 and errs[1] / errs[2] > 12, errs
    A_rbc, _ = rbc_area_volume()
    areas = []
    for n in (12, 24, 48):
        s = make_surface(RBC, n)
        _, wu = oracle.upsampled_surface(s.X, s.W, n, fine_pou(n))
        areas.append(abs(wu.sum() - A_rbc))
    assert areas[0] / areas[1] > 8 and areas[1] / areas[2] > 12, areas
    assert areas[1] < 1e-5 and areas[2] < 1e-6, areas


def test_downsample_of_upsample_converges_to_identity():
    """I_d I_u f -> f for a smooth density, at about fourth order."""
    import oracle
    from capsule_inputs import fine_grid
    errs = []
    for n in (8, 16, 32):
        s = make_surface(RBC, n)
        f = sh_force(s.x0, 4)
        tc, tf = fine_grid(n)
        back = oracle.spline_resample(oracle.spline_resample(f, n, tc, tf), 4 * n, tf, tc)
        errs.append(np.abs(back - f).max() / np.abs(f).max())
    assert errs[0] / errs[1] > 6 and errs[1] / errs[2] > 10 and errs[2] < 1e-5, errs


def test_upsampled_single_layer_on_the_sphere():
    """The whole sandwich on the unit sphere under uniform traction gives 2a f / (3 mu) at the
    nodes, converging under refinement."""
    import oracle
    from capsule_inputs import fine_pou
    errs = []
    for n in (6, 12):
        s = make_surface(SPHERE, n)
        f = np.tile([0.0, 0.0, 1.0], (s.N, 1))
        u = oracle.single_layer_upsampled(s.X, s.W, f, n, fine_pou(n), mu=1.0)
        errs.append(np.abs(u - [0.0, 0.0, 2.0 / 3.0]).max())
    assert errs[1] < 2e-5 and errs[1] < errs[0], errs


def test_upsampled_single_layer_of_normal_vanishes():
    """S[n] = 0 on a closed surface (the Stokeslet is divergence-free), through the whole
    upsampling step on the paper's a = 0.6 ellipsoid (Sec. 4.1 test shape), normalized by the
    response to e_z.  With delta_u = delta* of the fine grid (Sec. 3.4: delta_u by eq. (regparam)
    on the upsampled grid) the error is 2.3e-4 at n = 8 and 4.1e-5 at n = 12, falling at order
    about 4; a delta* taken from the coarse grid (4x larger, so about 4^5 times the O(delta^5)
    regularization error) gives 2.5e-2 and 6.3e-3 and fails both bounds."""
    import oracle
    from capsule_inputs import fine_pou
    errs = []
    for n in (8, 12):
        s = make_surface(ELLIPSOID_PAPER, n)
        psi = fine_pou(n)
        ez = np.tile([0.0, 0.0, 1.0], (s.N, 1))
        scale = np.abs(oracle.single_layer_upsampled(s.X, s.W, ez, n, psi)).max()
        errs.append(np.abs(oracle.single_layer_upsampled(s.X, s.W, s.normal, n, psi)).max() / scale)
    assert errs[0] < 5e-4 and errs[1] < 8e-5, errs
    assert math.log(errs[0] / errs[1]) / math.log(12 / 8) > 3.5, errs
