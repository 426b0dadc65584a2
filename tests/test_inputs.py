"""Pins for the synthetic inputs: grid, POU and trapezoid-POU weights (Sec. 3.1-3.3)."""
import math
import os

import numpy as np
import pytest
from scipy import integrate
from scipy.special import ellipeinc, ellipkinc

from capsule_inputs import (ELLIPSOID_PAPER, ELLIPSOID_SERVING, RBC, SPHERE, Shape, make_surface,
                            patch_centre, pou, real_sph_harm, sh_force)
from capsule_inputs.surfaces import R0_POU, RBC_C

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def ellipsoid_area(a, b, c):
    """Closed form (Legendre elliptic integrals) for the area of an ellipsoid."""
    a, b, c = sorted([a, b, c], reverse=True)
    if a == c:
        return 4 * math.pi * a * a
    phi = math.acos(c / a)
    m = (a * a * (b * b - c * c)) / (b * b * (a * a - c * c))
    s = math.sin(phi)
    return 2 * math.pi * c * c + 2 * math.pi * a * b / s * (ellipeinc(phi, m) * s * s
                                                             + ellipkinc(phi, m) * (1 - s * s))


def volume(surf):
    """V = integral of M . n with M = (x, 0, 0) (divergence theorem, Sec. 4.1 footnote)."""
    return float(np.sum(surf.w * surf.X[:, 0] * surf.normal[:, 0]))


def rbc_area_volume():
    """Area and volume of the biconcave shape as a surface of revolution (1-D quadrature)."""
    c0, c2, c4 = RBC_C

    def R(t):
        return math.sin(t)

    def Z(t):
        q = math.sin(t) ** 2
        return 0.5 * math.cos(t) * (c0 + c2 * q + c4 * q * q)

    def dR(t):
        return math.cos(t)

    def dZ(t):
        s, c = math.sin(t), math.cos(t)
        q = s * s
        P = c0 + c2 * q + c4 * q * q
        dP = (c2 + 2 * c4 * q) * 2 * s * c
        return 0.5 * (-s * P + c * dP)

    A = integrate.quad(lambda t: 2 * math.pi * R(t) * math.hypot(dR(t), dZ(t)), 0, math.pi,
                       epsabs=1e-13, epsrel=1e-12, limit=200)[0]
    V = integrate.quad(lambda t: -math.pi * R(t) ** 2 * dZ(t), 0, math.pi,
                       epsabs=1e-13, epsrel=1e-12, limit=200)[0]
    return A, V


def test_node_count_matches_paper_table():
    """N = 6 (m-1)^2 as printed in the ellipsoid table (Sec. 4.1)."""
    rows = np.loadtxt(os.path.join(GOLDEN, "tab_ellipsoid_sing_area_volume.txt"))
    for m, N, _, _ in rows:
        assert make_surface(SPHERE, int(m) - 1).N == int(N)


def test_pou_sums_to_one_and_support():
    rng = np.random.default_rng(0)
    x0 = rng.standard_normal((3, 20000))
    x0 /= np.linalg.norm(x0, axis=0)
    psi = pou(x0)
    assert np.allclose(psi.sum(axis=0), 1.0, atol=1e-14)
    assert np.all(psi >= 0)
    for i in range(6):
        d = np.arccos(np.clip(patch_centre(i + 1) @ x0, -1, 1))
        assert np.all(psi[i][d >= R0_POU] == 0.0)
        # support strictly inside the hemispherical patch
        assert np.all(psi[i][d >= math.pi / 2] == 0.0)


def test_patch_centres_are_the_six_axes():
    cs = np.array([patch_centre(i) for i in range(1, 7)])
    expect = np.array([[0, 1, 0], [0, -1, 0], [1, 0, 0], [-1, 0, 0], [0, 0, 1], [0, 0, -1]], float)
    assert np.allclose(cs, expect, atol=1e-15)


def test_nodes_lie_on_the_shape():
    s = make_surface(ELLIPSOID_SERVING, 20)
    a, b, c = ELLIPSOID_SERVING.axes
    lvl = (s.X[:, 0] / a) ** 2 + (s.X[:, 1] / b) ** 2 + (s.X[:, 2] / c) ** 2
    assert np.allclose(lvl, 1.0, atol=1e-14)
    s = make_surface(SPHERE, 20)
    assert np.allclose(np.linalg.norm(s.X, axis=1), 1.0, atol=1e-15)
    assert np.allclose(s.normal, s.X, atol=1e-14)


def test_sphere_area_and_volume_converge():
    for n, tol in [(31, 1e-5), (63, 1e-7)]:
        s = make_surface(SPHERE, n)
        assert abs(s.w.sum() - 4 * math.pi) / (4 * math.pi) < tol
        assert abs(volume(s) - 4 * math.pi / 3) / (4 * math.pi / 3) < tol


def test_ellipsoid_area_volume_beat_paper_table():
    """Analytic-W weights must be at least as accurate as the printed eps_A, eps_V."""
    rows = np.loadtxt(os.path.join(GOLDEN, "tab_ellipsoid_sing_area_volume.txt"))
    a, b, c = ELLIPSOID_PAPER.axes
    A_ex, V_ex = ellipsoid_area(a, b, c), 4 * math.pi * a * b * c / 3
    assert abs(A_ex - 9.389438372880) < 1e-10
    for m, N, epsA, epsV in rows:
        s = make_surface(ELLIPSOID_PAPER, int(m) - 1)
        assert abs(s.w.sum() - A_ex) / A_ex <= epsA
        assert abs(volume(s) - V_ex) / V_ex <= epsV


def test_serving_ellipsoid_and_rbc_weights():
    A_ex = ellipsoid_area(*ELLIPSOID_SERVING.axes)
    s = make_surface(ELLIPSOID_SERVING, 63)
    assert abs(s.w.sum() - A_ex) / A_ex < 1e-6
    A_rbc, V_rbc = rbc_area_volume()
    s = make_surface(RBC, 63)
    assert abs(s.w.sum() - A_rbc) / A_rbc < 1e-6
    assert abs(volume(s) - V_rbc) / V_rbc < 1e-6
    # the shape the workloads call "radius 1": rim at unit distance from the axis
    assert np.max(np.hypot(s.X[:, 0], s.X[:, 1])) <= 1.0 + 1e-15


def test_shifted_shape_is_a_translation():
    s0 = make_surface(RBC, 10)
    s1 = make_surface(Shape("rbc", shift=(3.0, -2.0, 1.0)), 10)
    assert np.allclose(s1.X - s0.X, [3.0, -2.0, 1.0], atol=1e-15)
    assert np.array_equal(s1.w, s0.w)


def test_real_harmonics_are_orthonormal():
    """Quadrature on a fine sphere: integral of Y_lm Y_l'm' = delta (POU trapezoid rule)."""
    s = make_surface(SPHERE, 47)
    lm = [(l, m) for l in range(5) for m in range(-l, l + 1)]
    Y = np.stack([real_sph_harm(l, m, s.x0) for l, m in lm], axis=1)
    G = (Y * s.w[:, None]).T @ Y
    assert np.allclose(G, np.eye(len(lm)), atol=1e-6)


def test_batched_harmonics_match_scipy_legendre():
    """The recurrence used for the force densities equals the scipy lpmv-based definition,
    including at the poles."""
    from capsule_inputs.forces import real_sph_harm_all
    s = make_surface(SPHERE, 9)
    x0 = np.concatenate([s.x0, [[0.0, 0.0, 1.0], [0.0, 0.0, -1.0]]])
    Y = real_sph_harm_all(x0, 8)
    k = 0
    for l in range(9):
        for m in range(-l, l + 1):
            assert np.allclose(Y[:, k], real_sph_harm(l, m, x0), atol=1e-12, rtol=1e-12)
            k += 1


def test_sh_force_is_seeded():
    s = make_surface(RBC, 8)
    assert np.array_equal(sh_force(s.x0, 7), sh_force(s.x0, 7))
    assert not np.array_equal(sh_force(s.x0, 7), sh_force(s.x0, 8))
