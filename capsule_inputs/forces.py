"""Seeded smooth force densities on a discretized surface.

The paper feeds the single layer the membrane force f = div_gamma(Lambda)
(Sec. 2, eq. (intf)); that force pipeline is not part of this build, so the
workloads use a synthetic smooth density instead: each Cartesian component is
a random real spherical-harmonic series of degree <= 8 evaluated at the node's
sphere pre-image x0, with coefficients c_lm ~ N(0, 1) / (l + 1)^2.

Convention: real orthonormal harmonics on S^2 (integral of Y_lm^2 over the
sphere is 1), Y_l0 = N_l0 P_l(cos t), Y_lm = sqrt(2) N_lm P_l^m(cos t) cos(m p)
for m > 0 and sqrt(2) N_l|m| P_l^|m|(cos t) sin(|m| p) for m < 0, with the
Condon-Shortley phase dropped. The coefficients are drawn per component in the
order l = 0..L, m = -l..l.
"""
from __future__ import annotations

import math

import numpy as np
from scipy.special import lpmv

L_MAX = 8


def real_sph_harm(l: int, m: int, x0: np.ndarray) -> np.ndarray:
    """Real orthonormal Y_lm at unit vectors x0 of shape (N, 3)."""
    ct = np.clip(x0[:, 2], -1.0, 1.0)
    ph = np.arctan2(x0[:, 1], x0[:, 0])
    am = abs(m)
    norm = math.sqrt((2 * l + 1) / (4 * math.pi)
                     * math.factorial(l - am) / math.factorial(l + am))
    P = lpmv(am, l, ct) * ((-1.0) ** am)   # undo scipy's Condon-Shortley phase
    if m == 0:
        return norm * P
    if m > 0:
        return math.sqrt(2.0) * norm * P * np.cos(am * ph)
    return math.sqrt(2.0) * norm * P * np.sin(am * ph)


def real_sph_harm_all(x0: np.ndarray, l_max: int = L_MAX) -> np.ndarray:
    """All real orthonormal Y_lm (same convention as real_sph_harm), shape (N, (l_max+1)^2),
    columns in the order l = 0..l_max, m = -l..l.

    Uses the three-term recurrence in l of Q_l^m = P_l^m(cos t) / sin^m t (no Condon-Shortley
    phase): Q_m^m = (2m-1)!!, Q_{m+1}^m = (2m+1) z Q_m^m,
    Q_l^m = ((2l-1) z Q_{l-1}^m - (l+m-1) Q_{l-2}^m) / (l-m), and sin^m t (cos m p, sin m p)
    = (Re, Im) (x + i y)^m, which is regular at the poles.
    """
    x, y, z = x0[:, 0], x0[:, 1], x0[:, 2]
    cm, sm = np.ones_like(x), np.zeros_like(x)       # Re, Im of (x + i y)^m
    out = np.empty(((l_max + 1) ** 2, x0.shape[0]))      # rows: contiguous writes
    col = lambda l, m: l * l + l + m
    dfact = 1.0
    for m in range(l_max + 1):
        if m > 0:
            dfact *= 2 * m - 1
            cm, sm = x * cm - y * sm, x * sm + y * cm
        q_prev, q = None, np.full(x.shape, dfact)
        for l in range(m, l_max + 1):
            if l == m + 1:
                q_prev, q = q, (2 * m + 1) * z * q
            elif l > m + 1:
                q_prev, q = q, ((2 * l - 1) * z * q - (l + m - 1) * q_prev) / (l - m)
            norm = math.sqrt((2 * l + 1) / (4 * math.pi)
                             * math.factorial(l - m) / math.factorial(l + m))
            if m == 0:
                out[col(l, 0)] = norm * q
            else:
                out[col(l, m)] = math.sqrt(2.0) * norm * q * cm
                out[col(l, -m)] = math.sqrt(2.0) * norm * q * sm
    return out.T


def sh_coefficients(seed: int, l_max: int = L_MAX) -> np.ndarray:
    """(3, (l_max+1)^2) coefficients c^k_lm ~ N(0,1)/(l+1)^2, seeded."""
    rng = np.random.default_rng(seed)
    scale = np.array([1.0 / (l + 1) ** 2 for l in range(l_max + 1) for _ in range(2 * l + 1)])
    return rng.standard_normal((3, scale.size)) * scale


def sh_force(x0: np.ndarray, seed: int, l_max: int = L_MAX) -> np.ndarray:
    """Force density (N, 3) from seeded SH coefficients, evaluated at pre-images x0."""
    c = sh_coefficients(seed, l_max)
    return np.ascontiguousarray(real_sph_harm_all(x0, l_max) @ c.T)


def uniform_force(N: int, f=(0.0, 0.0, 1.0)) -> np.ndarray:
    return np.tile(np.asarray(f, dtype=np.float64), (N, 1))
