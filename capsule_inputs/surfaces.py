"""Six-patch partition-of-unity surface discretizations (Sec. 3.1-3.3).

This module only builds *inputs*: node positions X, quadrature weights
w = psi * W * h^2, outward normals and the sphere pre-images x0 of the nodes.
It contains none of the single-layer arithmetic and is shared, unchanged, by
the CPU oracle tests and by the GPU path.

Paper references (Agarwal & Biros, "Numerical simulation of an extensible
capsule using regularized Stokes kernels and overset finite differences"):

* six hemispherical charts eta_i^0 on U = (0, pi)^2 ........ Sec. 3.1, eq. (param_maps)
* bump b(r) and POU psi_i^0, r0 = 5 pi / 12 ............... Sec. 3.1, eq. (pou0)
* POU pulled back through phi, frozen at t0 ................ Sec. 3.1 eq. (pou), Remark 1
* grid (j pi/m, k pi/m), j,k = 1..m-1, h_m = pi/m ........... Sec. 3.2, eq. (grid)
* ellipsoid map phi(x0) = (a x, b y, c z) .................. Sec. 3.2
* trapezoid-POU rule: weight psi W h^2 ..................... Sec. 3.3, eq. (smoothint)
* area element W = |x_u x x_v| ............................. Appendix B (differential formulas)

Readings where the paper is silent:

* "n x n points per patch" means m = n + 1, h = pi / (n + 1).
* W is evaluated from the analytic chart derivatives (the paper approximates the
  same quantity with its finite-difference scheme).
* The biconcave red-cell shape is not defined in the paper; it is the
  Evans-Fung profile z = +-1/2 sqrt(1 - q) (C0 + C2 q + C4 q^2), q = x^2 + y^2,
  realised by the smooth map phi(x, y, z) = (x, y, z (C0 + C2 q + C4 q^2) / 2).
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

R0_POU = 5.0 * np.pi / 12.0          # support radius of the bump, Sec. 3.1
RBC_C = (0.2072, 2.0026, -1.1228)    # Evans-Fung coefficients C0, C2, C4
N_PATCH = 6


# ----------------------------------------------------------------------------
# Charts eta_i^0 : (0, pi)^2 -> S^2 and their first derivatives.
# ----------------------------------------------------------------------------
def chart(i: int, u: np.ndarray, v: np.ndarray):
    """Return (x0, x0_u, x0_v), each of shape (3, ...), for chart i in 1..6."""
    su, cu, sv, cv = np.sin(u), np.cos(u), np.sin(v), np.cos(v)
    z = np.zeros_like(u)
    if i == 1:
        p = (su * cv, su * sv, cu)
        pu = (cu * cv, cu * sv, -su)
        pv = (-su * sv, su * cv, z)
    elif i == 2:
        p = (-su * cv, -su * sv, cu)
        pu = (-cu * cv, -cu * sv, -su)
        pv = (su * sv, -su * cv, z)
    elif i == 3:
        p = (su * sv, -su * cv, cu)
        pu = (cu * sv, -cu * cv, -su)
        pv = (su * cv, su * sv, z)
    elif i == 4:
        p = (-su * sv, su * cv, cu)
        pu = (-cu * sv, cu * cv, -su)
        pv = (-su * cv, -su * sv, z)
    elif i == 5:
        p = (su * cv, -cu, su * sv)
        pu = (cu * cv, su, cu * sv)
        pv = (-su * sv, z, su * cv)
    elif i == 6:
        p = (su * cv, cu, -su * sv)
        pu = (cu * cv, -su, -cu * sv)
        pv = (-su * sv, z, -su * cv)
    else:
        raise ValueError(f"chart index must be 1..6, got {i}")
    return np.array(p), np.array(pu), np.array(pv)


def patch_centre(i: int) -> np.ndarray:
    """eta_i^0(pi/2, pi/2): the point the bump of patch i is centred on."""
    x0, _, _ = chart(i, np.array(np.pi / 2), np.array(np.pi / 2))
    return x0


# ----------------------------------------------------------------------------
# Partition of unity, eq. (pou0).
# ----------------------------------------------------------------------------
def bump(r: np.ndarray) -> np.ndarray:
    """b(r) = exp(2 exp(-1/|r|) / (|r| - 1)) for |r| < 1, else 0."""
    a = np.abs(np.asarray(r, dtype=np.float64))
    out = np.zeros_like(a)
    inside = a < 1.0
    ai = a[inside]
    with np.errstate(divide="ignore", over="ignore", under="ignore"):
        e = np.where(ai > 0.0, np.exp(-1.0 / np.where(ai > 0, ai, 1.0)), 0.0)
        out[inside] = np.exp(2.0 * e / (ai - 1.0))
    return out


def great_circle(x0: np.ndarray, c: np.ndarray) -> np.ndarray:
    """Great-circle distance on S^2 between points x0 (3, ...) and a centre c (3,)."""
    dot = np.tensordot(c, x0, axes=(0, 0))
    return np.arccos(np.clip(dot, -1.0, 1.0))


def pou(x0: np.ndarray, r0: float = R0_POU) -> np.ndarray:
    """psi_i^0(x0) for all six patches; returns shape (6, ...)."""
    b = np.array([bump(great_circle(x0, patch_centre(i)) / r0) for i in range(1, 7)])
    return b / b.sum(axis=0)


# ----------------------------------------------------------------------------
# Diffeomorphisms phi : S^2 -> gamma (value and Jacobian at x0).
# ----------------------------------------------------------------------------
@dataclass(frozen=True)
class Shape:
    kind: str                      # "sphere", "ellipsoid", "rbc"
    axes: tuple = (1.0, 1.0, 1.0)  # ellipsoid semi-axes (a, b, c); sphere radius in axes[0]
    shift: tuple = (0.0, 0.0, 0.0)

    def map(self, x0: np.ndarray):
        """phi(x0) and the matrix D phi (3, 3, ...) of its R^3 extension."""
        x, y, z = x0
        one, zero = np.ones_like(x), np.zeros_like(x)
        if self.kind == "sphere":
            a = self.axes[0]
            X = a * x0
            J = np.array([[a * one, zero, zero], [zero, a * one, zero], [zero, zero, a * one]])
        elif self.kind == "ellipsoid":
            a, b, c = self.axes
            X = np.array([a * x, b * y, c * z])
            J = np.array([[a * one, zero, zero], [zero, b * one, zero], [zero, zero, c * one]])
        elif self.kind == "rbc":
            c0, c2, c4 = RBC_C
            q = x * x + y * y
            P = c0 + c2 * q + c4 * q * q
            dP = c2 + 2.0 * c4 * q
            X = np.array([x, y, 0.5 * z * P])
            J = np.array([[one, zero, zero], [zero, one, zero],
                          [z * x * dP, z * y * dP, 0.5 * P]])
        else:
            raise ValueError(self.kind)
        X = X + np.asarray(self.shift, dtype=np.float64).reshape((3,) + (1,) * (X.ndim - 1))
        return X, J


@dataclass
class Surface:
    """Nodes of the 6-patch discretization, in patch-major (i, j, k) order."""
    shape: Shape
    n: int                 # points per direction per patch (m = n + 1)
    h: float               # grid spacing pi / m
    X: np.ndarray          # (N, 3) node positions on gamma
    x0: np.ndarray         # (N, 3) pre-images on the unit sphere
    w: np.ndarray          # (N,)   psi * W * h^2
    psi: np.ndarray        # (N,)   own-patch POU value
    W: np.ndarray          # (N,)   area element |x_u x x_v|
    normal: np.ndarray     # (N, 3) outward unit normal
    patch: np.ndarray      # (N,)   patch index 1..6

    @property
    def N(self) -> int:
        return self.X.shape[0]


def make_surface(shape: Shape, n: int) -> Surface:
    """Discretize `shape` with 6 patches of n x n nodes (Sec. 3.2)."""
    if n < 1:
        raise ValueError("n must be >= 1")
    m = n + 1
    h = np.pi / m
    t = np.arange(1, m) * h
    U, V = np.meshgrid(t, t, indexing="ij")          # (j, k) row-major inside a patch
    Xs, x0s, ws, psis, Ws, ns, ps = [], [], [], [], [], [], []
    for i in range(1, N_PATCH + 1):
        p, pu, pv = chart(i, U, V)
        X, J = shape.map(p)
        xu = np.einsum("ab...,b...->a...", J, pu)
        xv = np.einsum("ab...,b...->a...", J, pv)
        cr = np.cross(xu, xv, axis=0)
        W = np.linalg.norm(cr, axis=0)
        nrm = cr / W
        # Orientation: the charts are right-handed w.r.t. the outward sphere
        # normal and every phi used here has det(D phi) > 0, so x_u x x_v points
        # outward. Checked rather than assumed: the pushed-forward sphere normal is
        # det(J) J^{-T} x0 = ((J2 x J3).x0, (J3 x J1).x0, (J1 x J2).x0), J_k the rows of J.
        r1, r2, r3 = J[0], J[1], J[2]
        push = np.array([np.einsum("a...,a...->...", np.cross(r2, r3, axis=0), p),
                         np.einsum("a...,a...->...", np.cross(r3, r1, axis=0), p),
                         np.einsum("a...,a...->...", np.cross(r1, r2, axis=0), p)])
        det = np.einsum("a...,a...->...", r1, np.cross(r2, r3, axis=0))
        if np.any(det <= 0) or np.any(np.einsum("a...,a...->...", nrm, push) <= 0):
            raise RuntimeError("chart orientation is not outward")
        psi = pou(p)[i - 1]
        Xs.append(X.reshape(3, -1).T)
        x0s.append(p.reshape(3, -1).T)
        Ws.append(W.ravel())
        psis.append(psi.ravel())
        ws.append((psi * W * h * h).ravel())
        ns.append(nrm.reshape(3, -1).T)
        ps.append(np.full(n * n, i, dtype=np.int32))
    return Surface(shape=shape, n=n, h=h,
                   X=np.ascontiguousarray(np.concatenate(Xs)),
                   x0=np.ascontiguousarray(np.concatenate(x0s)),
                   w=np.concatenate(ws), psi=np.concatenate(psis), W=np.concatenate(Ws),
                   normal=np.ascontiguousarray(np.concatenate(ns)),
                   patch=np.concatenate(ps))


SPHERE = Shape("sphere")
RBC = Shape("rbc")
ELLIPSOID_SERVING = Shape("ellipsoid", (1.0, 0.8, 0.5))   # axes 1 : 0.8 : 0.5
ELLIPSOID_PAPER = Shape("ellipsoid", (0.6, 1.0, 1.0))     # Sec. 4.1 test shape


def fine_grid(n: int, factor: int = 4):
    """Parameters of the upsampled grid of a patch with n x n nodes: factor * n nodes per
    direction at j pi / (factor n + 1), j = 1..factor n (N_up = factor^2 N, the count of the
    paper's upsampling table), and the coarse parameters j pi / (n + 1), j = 1..n."""
    nf = factor * n
    return (np.arange(1, n + 1) * np.pi / (n + 1), np.arange(1, nf + 1) * np.pi / (nf + 1))


def fine_pou(n: int, factor: int = 4) -> np.ndarray:
    """Own-patch POU values at the upsampled nodes (patch-major, row-major), eq. (pou) at the
    sphere pre-images: the precomputed Psi_u of the upsampling step (Sec. 3.4)."""
    _, tf = fine_grid(n, factor)
    U, V = np.meshgrid(tf, tf, indexing="ij")
    out = []
    for i in range(1, N_PATCH + 1):
        p, _, _ = chart(i, U, V)
        out.append(pou(p)[i - 1].ravel())
    return np.concatenate(out)


def fine_positions(shape: "Shape", n: int, factor: int = 4) -> np.ndarray:
    """Exact surface positions at the upsampled nodes (for checking interpolation only)."""
    _, tf = fine_grid(n, factor)
    U, V = np.meshgrid(tf, tf, indexing="ij")
    out = []
    for i in range(1, N_PATCH + 1):
        p, _, _ = chart(i, U, V)
        X, _ = shape.map(p)
        out.append(X.reshape(3, -1).T)
    return np.ascontiguousarray(np.concatenate(out))
