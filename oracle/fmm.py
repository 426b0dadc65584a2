"""Single-level kernel-independent FMM of the single layer (Sec. 5, "Fast multipole method based
acceleration"): plain FP64 reference.  TEST INFRASTRUCTURE ONLY -- used by the tests and the
benchmark's error figures, never by the product path, and sharing no code with the GPU library.

The paper's three steps, in its order:

1. k-means clustering of the discretization points into k clusters (the paper takes k = 100).
2. Each cluster is enclosed by a cube, the equivalent surface, with equivalent sources on a
   regular grid of its boundary, and by a larger cube, the check surface, carrying a grid of check
   points.  The densities of the equivalent sources are fitted so that they reproduce, on the check
   surface, the potential of the cluster's own sources.
3. Targets in neighbouring clusters are summed directly (the regularized kernel of eq. (regstokes));
   targets in the other clusters take the cluster's equivalent sources.

Readings (the paper gives no further detail; each is a choice recorded here):

* k-means: Lloyd's iteration from the points at indices floor(j N / k), j = 0..k-1, of the input
  order; a point joins the nearest centroid (squared distance ((dx dx + dy dy) + dz dz), ties to
  the lower index); it stops at the first assignment that changes no label, after at most
  `max_iter` assignments.  Centroid sums are exact: each coordinate is quantized to an integer
  q = rint((x - lo) 2^(24 - e)) (lo the smallest coordinate of that axis, 2^e >= the largest axis
  extent), summed in 64-bit integers, and the centroid is lo + (sum / count) 2^(e - 24).  An empty
  cluster keeps its centroid.  (Exact sums make the clustering independent of summation order.)
* Cubes: the box of cluster S has centre o_S = (lo + hi) / 2 of its points' bounding box and half
  width a_S = max over axes of (hi - lo) / 2 (at least 2^-20 of the largest axis extent of all
  points).  Equivalent surface: half width 1.05 a_S; check surface: 2.95 a_S (the kernel-independent
  FMM's usual upward-pass radii); grid: the p x p x p lattice of the cube's boundary, p points per
  edge, N_eq = p^3 - (p - 2)^3 points (p = 5, 6, 8 give 98, 152, 296 against the paper's 96, 128,
  256).
* Neighbours: cluster T is near S when T == S, when T's box meets the cube of half width 3 a_S
  around o_S, or when the gap between the two boxes is below 6.9 delta_T (delta_T the largest delta
  of T's points).  Far targets are therefore outside S's check surface, and every far pair has
  r >= 6.9 delta, where the smoothing factors equal 1 in double precision: the far field uses the
  plain Stokeslet (`oracle.stokeslet`).
* Fit: the check potentials v_c = sum_{j in S} G(c - y_j) g_j (g = w f, G the plain Stokeslet);
  the equivalent densities phi minimize |K phi - v_c|^2 + lambda |phi|^2 with K = G(check -
  equivalent) and lambda = 1e-8 times the largest squared column norm of K (Tikhonov).  G is
  homogeneous of degree -1, so K = K_unit / a_S and phi = a_S M_unit v_c with one operator M_unit of
  the unit cube, computed here with numpy's least-squares solver.
"""
from __future__ import annotations

import math

import numpy as np

ALPHA_EQ = 1.05        # equivalent surface / cluster box
ALPHA_CHECK = 2.95     # check surface / cluster box
ALPHA_FAR = 3.0        # targets beyond this cube around a cluster take its equivalent sources
TIKHONOV = 1e-8        # lambda / largest squared column norm of the check-from-equivalent matrix
RHO_EXACT = 6.9        # s1 = s2 = 1 to double precision beyond r / delta = 6.9
KMEANS_MAX_ITER = 100


def quantize(X):
    """(lo, scale, Q): per-axis minimum, the power of two 2^(24 - e), and the integer coordinates."""
    X = np.asarray(X, dtype=np.float64)
    lo = X.min(axis=0)
    ext = float((X.max(axis=0) - lo).max())
    e = math.frexp(ext)[1] if ext > 0.0 else 0        # ext < 2^e
    scale = math.ldexp(1.0, 24 - e)
    Q = np.rint((X - lo) * scale).astype(np.int64)
    return lo, scale, Q


def kmeans(X, k, max_iter=KMEANS_MAX_ITER):
    """Labels (N,) int32, centroids (k, 3) and the number of assignments made."""
    X = np.asarray(X, dtype=np.float64)
    N = X.shape[0]
    lo, scale, Q = quantize(X)
    C = X[(np.arange(k, dtype=np.int64) * N) // k].copy()
    labels = None
    it = 0
    for it in range(1, max_iter + 1):
        new = np.empty(N, dtype=np.int32)
        for s in range(0, N, 65536):
            dx = X[s:s + 65536, None, 0] - C[None, :, 0]
            dy = X[s:s + 65536, None, 1] - C[None, :, 1]
            dz = X[s:s + 65536, None, 2] - C[None, :, 2]
            d2 = (dx * dx + dy * dy) + dz * dz
            new[s:s + 65536] = np.argmin(d2, axis=1)     # first minimum: the lower index
        if labels is not None and np.array_equal(new, labels):
            break
        labels = new
        counts = np.bincount(labels, minlength=k)
        for c in range(3):
            # integer coordinates below 2^24, at most 2^28 points: every partial sum is an integer
            # below 2^53, so the double-precision bincount is exact whatever its order
            sums = np.bincount(labels, weights=Q[:, c], minlength=k).astype(np.int64)
            has = counts > 0
            C[has, c] = lo[c] + (sums[has].astype(np.float64) / counts[has].astype(np.float64)) / scale
    return labels, C, it


def boxes(X, labels, k):
    """Per cluster: centre (k, 3), half width (k,), point count (k,)."""
    X = np.asarray(X, dtype=np.float64)
    ext = float((X.max(axis=0) - X.min(axis=0)).max())
    amin = math.ldexp(ext, -20)
    o = np.zeros((k, 3))
    a = np.zeros(k)
    cnt = np.bincount(labels, minlength=k)
    for j in range(k):
        if cnt[j] == 0:
            continue
        P = X[labels == j]
        lo, hi = P.min(axis=0), P.max(axis=0)
        o[j] = 0.5 * (lo + hi)
        a[j] = max(0.5 * float((hi - lo).max()), amin)
    return o, a, cnt


def near_mask(o, a, cnt, dmax):
    """near[T, S] for non-empty clusters T, S (dmax[T]: the largest delta of T's points)."""
    k = len(a)
    near = np.zeros((k, k), dtype=bool)
    for T in range(k):
        if cnt[T] == 0:
            continue
        for S in range(k):
            if cnt[S] == 0:
                continue
            d = np.abs(o[T] - o[S])
            meets = bool(np.all(d <= a[T] + ALPHA_FAR * a[S]))
            g = np.maximum(d - (a[T] + a[S]), 0.0)
            gap = math.sqrt((g[0] * g[0] + g[1] * g[1]) + g[2] * g[2])
            near[T, S] = T == S or meets or gap < RHO_EXACT * dmax[T]
    return near


def cube_points(p):
    """The p^3 - (p - 2)^3 lattice points on the boundary of [-1, 1]^3, lexicographic (i, j, l)."""
    g = np.array([-1.0 + 2.0 * i / (p - 1) for i in range(p)])
    pts = [(g[i], g[j], g[l]) for i in range(p) for j in range(p) for l in range(p)
           if i in (0, p - 1) or j in (0, p - 1) or l in (0, p - 1)]
    return np.array(pts)


def stokeslet_matrix(T, S):
    """(3 n_T, 3 n_S) matrix of the plain Stokeslet, component-major blocks: row a n_T + i, column
    b n_S + j holds delta_ab / r + d_a d_b / r^3, d = T_i - S_j."""
    d = T[:, None, :] - S[None, :, :]
    r = np.sqrt((d * d).sum(axis=2))
    nT, nS = T.shape[0], S.shape[0]
    K = np.zeros((3 * nT, 3 * nS))
    for a in range(3):
        for b in range(3):
            K[a * nT:(a + 1) * nT, b * nS:(b + 1) * nS] = (a == b) / r + d[:, :, a] * d[:, :, b] / r ** 3
    return K


def unit_operator(p):
    """M_unit (3 N_eq, 3 N_eq): Tikhonov least-squares map from check potentials to equivalent
    densities for the unit box (equivalent surface 1.05, check surface 2.95 times the half width)."""
    E = cube_points(p)
    K = stokeslet_matrix(ALPHA_CHECK * E, ALPHA_EQ * E)
    lam = TIKHONOV * float((K * K).sum(axis=0).max())
    n = K.shape[1]
    A = np.vstack([K, math.sqrt(lam) * np.eye(n)])
    B = np.vstack([np.eye(K.shape[0]), np.zeros((n, K.shape[0]))])
    return np.linalg.lstsq(A, B, rcond=None)[0]


def single_layer_fmm(X, w, f, delta, mu=1.0, delta_tgt=None, k=100, p=6, max_iter=KMEANS_MAX_ITER,
                     nthreads=0, details=False, only=None):
    """u (N, 3) at the nodes X by the single-level FMM (targets = sources).  With details=True also
    returns a dict with the labels, boxes, neighbour mask and the near and far parts.  `only`: an
    iterable of cluster indices whose targets are evaluated (the others are NaN) -- the clustering
    and every cluster's equivalent sources are computed in full either way."""
    import oracle
    X = np.asarray(X, dtype=np.float64)
    f = np.asarray(f, dtype=np.float64)
    w = np.asarray(w, dtype=np.float64)
    N = X.shape[0]
    dt = np.full(N, float(delta)) if delta_tgt is None else np.asarray(delta_tgt, dtype=np.float64)
    labels, C, iters = kmeans(X, k, max_iter)
    o, a, cnt = boxes(X, labels, k)
    dmax = np.zeros(k)
    np.maximum.at(dmax, labels, dt)
    near = near_mask(o, a, cnt, dmax)
    g = w[:, None] * f
    E = cube_points(p)
    M = unit_operator(p)
    ne = E.shape[0]
    members = [np.flatnonzero(labels == j) for j in range(k)]
    # step 2: equivalent densities of every cluster
    eq_pts, eq_g = [None] * k, [None] * k
    for S in range(k):
        if cnt[S] == 0:
            continue
        chk = o[S] + ALPHA_CHECK * a[S] * E
        v = oracle.stokeslet(X[members[S]], g[members[S]], chk, nthreads=nthreads)
        phi = a[S] * (M @ np.concatenate([v[:, 0], v[:, 1], v[:, 2]]))
        eq_pts[S] = o[S] + ALPHA_EQ * a[S] * E
        eq_g[S] = np.stack([phi[:ne], phi[ne:2 * ne], phi[2 * ne:]], axis=1)
    # step 3: near field directly, far field from the equivalent sources
    scale = 1.0 / (8.0 * math.pi * mu)
    u_near = np.zeros((N, 3))
    u_far = np.zeros((N, 3))
    if only is not None:
        u_near[:] = np.nan
    for T in (range(k) if only is None else only):
        if cnt[T] == 0:
            continue
        u_far[members[T]] = 0.0
        tg = members[T]
        nb = [S for S in range(k) if cnt[S] and near[T, S]]
        fr = [S for S in range(k) if cnt[S] and not near[T, S]]
        src = np.concatenate([members[S] for S in nb])
        u_near[tg] = oracle.single_layer(X[src], w[src], f[src], 0.0, mu=mu, targets=X[tg],
                                         delta_tgt=dt[tg], nthreads=nthreads)
        if fr:
            Y = np.concatenate([eq_pts[S] for S in fr])
            G = np.concatenate([eq_g[S] for S in fr])
            u_far[tg] = scale * oracle.stokeslet(Y, G, X[tg], nthreads=nthreads)
    u = u_near + u_far
    if details:
        return u, {"labels": labels, "centroids": C, "iterations": iters, "centre": o,
                   "half_width": a, "count": cnt, "near": near, "u_near": u_near, "u_far": u_far}
    return u
