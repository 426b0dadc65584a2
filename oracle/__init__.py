"""CPU FP64 oracle for the regularized Stokes single layer.

TEST INFRASTRUCTURE ONLY.  Imported by the tests, by the smoke check and by the
benchmark's CPU-baseline leg; the product library never imports or links it and
shares no code with it.  The arithmetic lives in ``slref.c`` (plain C, glibc
erf/exp, Neumaier sums, OpenMP over targets); this module only builds and loads
it and marshals numpy arrays.

Also the per-patch regularization parameter of eq. (regparam) (``patch_delta``) and the
upsampling step around the sum (``single_layer_upsampled``: X, F and the area element W
upsampled by per-patch cubic splines, the sum on the fine grid with delta_u, the spline back).

Pinned by ``tests/test_oracle_pins.py`` against the r -> 0 limits stated in
Sec. 3.4, vanishing moments of s - 1, the sphere's closed-form drag and
rotation velocities, S[n] = 0 with the O(delta^5) order, the discrete
reciprocity identity, translation/rotation invariance and a 40-digit brute
force on tiny inputs; the upsampling step by exact bicubic reproduction of
positions, derivatives and fine weights, fourth-order convergence of the fine
nodes and of the fine weights' area, the sphere's closed form through the whole
step, and S[n] = 0 through the whole step at a bound that a coarse-grid delta
fails.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "slref.c")
# SLREF_LIB names another build of slref.c to load (the sanitizer test uses it).
LIB_PATH = os.environ.get("SLREF_LIB") or os.path.join(_HERE, "libslref.so")

_lib = None


def build(force: bool = True) -> str:
    """Compile slref.c into libslref.so next to it (gcc -O2 -fopenmp, no fast-math)."""
    if force or not os.path.exists(LIB_PATH):
        tmp = LIB_PATH + f".tmp{os.getpid()}"
        cmd = ["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared",
               "-fno-fast-math", "-Wall", "-Wextra", "-o", tmp, _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, LIB_PATH)
    return LIB_PATH


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build(force=False)
        lib = ctypes.CDLL(LIB_PATH)
        P = ctypes.POINTER(ctypes.c_double)
        i64, d = ctypes.c_int64, ctypes.c_double
        lib.slref_eval.argtypes = [i64, P, P, P, P, P, P, P, i64, P, P, P, d, P, d, P, P, P,
                                   ctypes.c_int]
        lib.slref_eval.restype = ctypes.c_int
        lib.slref_smoothing.argtypes = [d, P, P]
        lib.slref_smoothing.restype = None
        lib.slref_kernel.argtypes = [d, d, P, P]
        lib.slref_kernel.restype = None
        lib.slref_patch_delta.argtypes = [i64, i64, P, P, P, d, P]
        lib.slref_patch_delta.restype = ctypes.c_int
        lib.slref_stokeslet.argtypes = [i64, P, P, P, P, P, P, i64, P, P, P, P, P, P, ctypes.c_int]
        lib.slref_stokeslet.restype = ctypes.c_int
        lib.slref_max_threads.argtypes = []
        lib.slref_max_threads.restype = ctypes.c_int
        _lib = lib
    return _lib


def _ptr(a):
    if a is None:
        return None
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _col(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def single_layer(X, w, f, delta, mu=1.0, targets=None, delta_tgt=None, nthreads=0):
    """u (n_tgt, 3) at `targets` (default: the source nodes X) from sources X (N, 3),
    weights w (N,), density f (N, 3)."""
    lib = _load()
    X = np.asarray(X, dtype=np.float64)
    f = np.asarray(f, dtype=np.float64)
    sx, sy, sz = _col(X[:, 0]), _col(X[:, 1]), _col(X[:, 2])
    fx, fy, fz = _col(f[:, 0]), _col(f[:, 1]), _col(f[:, 2])
    w = _col(w)
    if targets is None:
        nt = X.shape[0]
        tx = ty = tz = None
    else:
        T = np.asarray(targets, dtype=np.float64).reshape(-1, 3)
        nt = T.shape[0]
        tx, ty, tz = _col(T[:, 0]), _col(T[:, 1]), _col(T[:, 2])
    dt = None if delta_tgt is None else _col(delta_tgt)
    if dt is not None and dt.shape[0] != nt:
        raise ValueError("delta_tgt must have one entry per target")
    ux, uy, uz = (np.zeros(nt) for _ in range(3))
    rc = lib.slref_eval(X.shape[0], _ptr(sx), _ptr(sy), _ptr(sz), _ptr(w), _ptr(fx), _ptr(fy),
                        _ptr(fz), nt, _ptr(tx), _ptr(ty), _ptr(tz), float(delta), _ptr(dt),
                        float(mu), _ptr(ux), _ptr(uy), _ptr(uz), int(nthreads))
    if rc != 0:
        raise ValueError("slref_eval rejected its arguments")
    return np.stack([ux, uy, uz], axis=1)


def stokeslet(Y, g, targets, nthreads=0):
    """Plain Stokeslet sum v (n_tgt, 3) = sum_j [g_j / r + (g_j . d) d / r^3], d = t - y_j, from
    sources Y (N, 3) with densities g (N, 3) (no weights, no 1/(8 pi mu); r = 0 pairs skipped)."""
    lib = _load()
    Y = np.asarray(Y, dtype=np.float64).reshape(-1, 3)
    g = np.asarray(g, dtype=np.float64).reshape(-1, 3)
    T = np.asarray(targets, dtype=np.float64).reshape(-1, 3)
    cols = [_col(Y[:, 0]), _col(Y[:, 1]), _col(Y[:, 2]), _col(g[:, 0]), _col(g[:, 1]),
            _col(g[:, 2]), _col(T[:, 0]), _col(T[:, 1]), _col(T[:, 2])]
    out = [np.zeros(T.shape[0]) for _ in range(3)]
    rc = lib.slref_stokeslet(Y.shape[0], *[_ptr(c) for c in cols[:6]], T.shape[0],
                             *[_ptr(c) for c in cols[6:]], *[_ptr(o) for o in out], int(nthreads))
    if rc != 0:
        raise ValueError("slref_stokeslet rejected its arguments")
    return np.stack(out, axis=1)


def patch_delta(X, n, C=1.0):
    """Per-node delta = C delta*_i of eq. (regparam) for nodes X (6 n^2, 3) in patch-major,
    row-major (l, l') order, n x n nodes per patch."""
    lib = _load()
    X = np.asarray(X, dtype=np.float64).reshape(-1, 3)
    if n < 1 or X.shape[0] % (n * n) != 0:
        raise ValueError("X must hold whole patches of n x n nodes")
    n_patches = X.shape[0] // (n * n)
    out = np.zeros(X.shape[0])
    rc = lib.slref_patch_delta(n_patches, int(n), _ptr(_col(X[:, 0])), _ptr(_col(X[:, 1])),
                               _ptr(_col(X[:, 2])), float(C), _ptr(out))
    if rc != 0:
        raise ValueError("slref_patch_delta rejected its arguments")
    return out


# ----------------------------------------------------------------------------------------------
# Upsampling step (Sec. 3.4, "Upsampling"; the right-hand-side algorithm of Sec. 3.6, its
# upsampling, single-layer and downsampling steps): u = I_d S^{delta_u}[I_u f] on X_u = I_u X.
# The algorithm upsamples the nodes, the density and the area element with the same operator
# (X_u = I_u X, F_u = I_u F, W_u = I_u W) and sums with X_u, F_u, the precomputed POU values
# Psi_u and W_u, i.e. with the trapezoid-POU weights w_u = psi_u W_u h_u^2 of eq. (smoothint) on
# the fine grid.  Readings: the fine grid has factor*n nodes per direction at j pi/(factor n + 1)
# (N_up = factor^2 N, the count of the paper's table); I_u and I_d are per-patch tensor-product
# cubic splines with not-a-knot ends (de Boor's default), the end pieces extended where the fine
# grid reaches past the coarse nodes; delta_u is eq. (regparam) on the fine grid.
# ----------------------------------------------------------------------------------------------
def _grids(n, factor):
    nf = factor * n
    return np.arange(1, n + 1) * np.pi / (n + 1), np.arange(1, nf + 1) * np.pi / (nf + 1)


def spline_resample(F, n_from, t_from, t_to, du=0, dv=0):
    """Per patch, the tensor-product not-a-knot cubic spline through values F on the grid
    t_from x t_from (patch-major, row-major, trailing components allowed), evaluated (or its
    du-th u- and dv-th v-derivative) on t_to x t_to."""
    from scipy.interpolate import CubicSpline
    F = np.asarray(F, dtype=np.float64)
    comp = F.shape[1:]
    G = F.reshape((-1, n_from, n_from) + comp)
    a = CubicSpline(t_from, G, axis=1, bc_type="not-a-knot", extrapolate=True)
    G = a(t_to, du) if du else a(t_to)
    b = CubicSpline(t_from, G, axis=2, bc_type="not-a-knot", extrapolate=True)
    G = b(t_to, dv) if dv else b(t_to)
    return G.reshape((-1,) + comp)


def upsampled_surface(X, W, n, psi_up, factor=4):
    """(X_u, w_u) on the fine grid from the coarse nodes X (N, 3) and their area elements W (N,):
    X_u = I_u X, W_u = I_u W, w_u = psi_u W_u h_u^2."""
    tc, tf = _grids(n, factor)
    Xu = spline_resample(X, n, tc, tf)
    Wu = spline_resample(np.asarray(W, dtype=np.float64), n, tc, tf)
    hf = np.pi / (factor * n + 1)
    return Xu, np.asarray(psi_up, dtype=np.float64) * Wu * hf * hf


def single_layer_upsampled(X, W, f, n, psi_up, mu=1.0, C=1.0, factor=4, nthreads=0):
    """u at the coarse nodes: I_d S^{delta_u}[I_u f] evaluated on the upsampled surface, from the
    coarse nodes X, area elements W and density f."""
    tc, tf = _grids(n, factor)
    Xu, wu = upsampled_surface(X, W, n, psi_up, factor)
    fu = spline_resample(f, n, tc, tf)
    du = patch_delta(Xu, factor * n, C=C)
    uu = single_layer(Xu, wu, fu, 0.0, mu=mu, delta_tgt=du, nthreads=nthreads)
    return spline_resample(uu, factor * n, tf, tc)


def smoothing(p: float):
    """(s1(p), s2(p)) as printed in Sec. 3.4."""
    lib = _load()
    a, b = ctypes.c_double(), ctypes.c_double()
    lib.slref_smoothing(float(p), ctypes.byref(a), ctypes.byref(b))
    return a.value, b.value


def kernel(r: float, delta: float):
    """(s1(r/delta)/r, s2(r/delta)/r^3), with the r = 0 limits."""
    lib = _load()
    a, b = ctypes.c_double(), ctypes.c_double()
    lib.slref_kernel(float(r), float(delta), ctypes.byref(a), ctypes.byref(b))
    return a.value, b.value


def max_threads() -> int:
    return int(_load().slref_max_threads())


def rel_inf_error(u, u_ref) -> float:
    """eps = ||u - u_ref||_inf / ||u_ref||_inf over all targets and components (Sec. 4.1)."""
    u, u_ref = np.asarray(u), np.asarray(u_ref)
    return float(np.max(np.abs(u - u_ref)) / np.max(np.abs(u_ref)))
