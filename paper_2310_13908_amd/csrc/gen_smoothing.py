#!/usr/bin/env python3
"""Generate sl_smoothing_coeffs.h: constants of the device evaluation of the smoothing factors
s1, s2 of Sec. 3.4 (s1(p) = erf p - (2/3) p (2p^2 - 5) e^{-p^2}/sqrt(pi),
s2(p) = erf p - (2/3) p (4p^4 - 14p^2 + 3) e^{-p^2}/sqrt(pi)).

The device code splits the regularized zone p = r/delta < 6.9 in two:

* p^2 < 0.25: power series in q = p^2 of F1 = s1(p)/p and F2 = s2(p)/p^3, obtained by
  expanding erf and exp term by term:
      sqrt(pi) F1(q) = sum_n (-1)^n 8 (n+1)(n+2) q^n / (3 (2n+1) n!)
      sqrt(pi) F2(q) = sum_n (-1)^n 16 (n+2)(n+3) q^n / (3 (2n+3) n!)
  (F1(0) = 16/(3 sqrt(pi)), F2(0) = 32/(3 sqrt(pi)): the r -> 0 limits of Sec. 3.4).
* 0.5 <= p < 6.9: s = 1 - e^{-q} (g(p) + P(p)) with the exact polynomial parts
  P1 = (2/3)p(2q-5)/sqrt(pi), P2 = (2/3)p(4q^2-14q+3)/sqrt(pi) and the scaled complementary
  error function g(p) = e^{p^2} erfc(p), approximated by a polynomial in t = 3/(3+p)
  interpolated at Chebyshev nodes with 40-digit mpmath values; e^{-q} uses its Taylor
  series after reduction by powers of two.

Run: python gen_smoothing.py  (rewrites sl_smoothing_coeffs.h next to this file and prints the
achieved double-precision error of every approximation).
"""
from __future__ import annotations

import math
import os
import struct

import mpmath as mp
import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
OUT = os.path.join(HERE, "sl_smoothing_coeffs.h")

SERIES_Q_MAX = 0.25     # series used for q = p^2 below this
SERIES_TERMS = 14
G_LO, G_HI = 0.5, 6.9   # range of the g fit (p)
G_K = 3.0               # t = G_K / (G_K + p)
G_DEG = 16
EXP_DEG = 13            # Taylor degree of e^x on |x| <= ln2/2
# Single-precision smoothing of the mixed path (0.5 <= p < 5): g as a polynomial in
# t - G32_MID, t = G_K / (G_K + p), coefficients rounded to single precision.
G32_LO, G32_HI = 0.5, 5.0
G32_DEG = 7


def series_coeffs():
    sp = mp.sqrt(mp.pi)
    c1 = [(-1) ** n * mp.mpf(8 * (n + 1) * (n + 2)) / (3 * (2 * n + 1) * mp.factorial(n)) / sp
          for n in range(SERIES_TERMS)]
    c2 = [(-1) ** n * mp.mpf(16 * (n + 2) * (n + 3)) / (3 * (2 * n + 3) * mp.factorial(n)) / sp
          for n in range(SERIES_TERMS)]
    return c1, c2


def g_exact(p):
    p = mp.mpf(p)
    return mp.exp(p * p) * mp.erfc(p)


def g_coeffs():
    ta, tb = G_K / (G_K + G_HI), G_K / (G_K + G_LO)
    nodes = [mp.cos(mp.pi * (j + mp.mpf(1) / 2) / (G_DEG + 1)) for j in range(G_DEG + 1)]
    ts = [(ta + tb) / 2 + (tb - ta) / 2 * c for c in nodes]
    A = mp.matrix([[t ** i for i in range(G_DEG + 1)] for t in ts])
    y = mp.matrix([g_exact(G_K / t - G_K) for t in ts])
    return [c for c in mp.lu_solve(A, y)]


def g32_coeffs():
    ta, tb = G_K / (G_K + G32_HI), G_K / (G_K + G32_LO)
    mid = float(np.float32((ta + tb) / 2))
    nodes = [mp.cos(mp.pi * (j + mp.mpf(1) / 2) / (G32_DEG + 1)) for j in range(G32_DEG + 1)]
    ts = [mp.mpf((ta + tb) / 2) + mp.mpf((tb - ta) / 2) * c for c in nodes]
    A = mp.matrix([[(t - mp.mpf(mid)) ** i for i in range(G32_DEG + 1)] for t in ts])
    y = mp.matrix([g_exact(G_K / t - G_K) for t in ts])
    cf = [float(np.float32(float(c))) for c in mp.lu_solve(A, y)]
    # error of the single-precision evaluation (numpy float32 mirrors the device arithmetic)
    p = np.linspace(G32_LO, G32_HI, 2001)
    t = (np.float32(G_K) * (np.float32(1) / (np.float32(G_K) + p.astype(np.float32)))).astype(np.float32)
    t = (t - np.float32(mid)).astype(np.float32)
    v = np.full_like(t, np.float32(cf[-1]))
    for c in cf[-2::-1]:
        v = (v * t + np.float32(c)).astype(np.float32)
    err = max(float(abs(mp.mpf(float(a)) - g_exact(float(x)))) for x, a in zip(p[::4], v[::4]))
    return cf, mid, err


def horner(cf, x):
    p = np.full_like(x, float(cf[-1]))
    for c in cf[-2::-1]:
        p = p * x + float(c)
    return p


def s_exact(p):
    p = mp.mpf(p)
    e = mp.exp(-p * p) / mp.sqrt(mp.pi)
    return (mp.erf(p) - mp.mpf(2) / 3 * p * (2 * p * p - 5) * e,
            mp.erf(p) - mp.mpf(2) / 3 * p * (4 * p ** 4 - 14 * p * p + 3) * e)


def ln2_split():
    ln2 = float(mp.log(2))
    bits = struct.unpack("<Q", struct.pack("<d", ln2))[0] & ~((1 << 32) - 1)
    hi = struct.unpack("<d", struct.pack("<Q", bits))[0]
    lo = float(mp.log(2) - mp.mpf(hi))
    return hi, lo


def check(c1, c2, gc):
    """Max errors of the double-precision evaluation (numpy mirrors the device arithmetic)."""
    mp.mp.dps = 40
    rep = {}
    q = np.linspace(0.0, SERIES_Q_MAX, 2001)
    F1 = horner(c1, q)
    F2 = horner(c2, q)
    e1 = e2 = 0.0
    for qi, a, b in zip(q[::10], F1[::10], F2[::10]):
        p = mp.sqrt(mp.mpf(float(qi)))
        if p == 0:
            r1, r2 = 16 / (3 * mp.sqrt(mp.pi)), 32 / (3 * mp.sqrt(mp.pi))
        else:
            s1, s2 = s_exact(p)
            r1, r2 = s1 / p, s2 / p ** 3
        e1 = max(e1, float(abs(a - r1) / r1))
        e2 = max(e2, float(abs(b - r2) / r2))
    rep["series_rel_F1"], rep["series_rel_F2"] = e1, e2
    p = np.linspace(G_LO, G_HI, 3001)
    gv = horner(gc, G_K / (G_K + p))
    rep["g_abs"] = max(float(abs(mp.mpf(float(a)) - g_exact(float(x)))) for x, a in zip(p[::3], gv[::3]))
    return rep


def fmt(v):
    return f"{float(v):.17e}"


def main():
    mp.mp.dps = 40
    c1, c2 = series_coeffs()
    gc = g_coeffs()
    hi, lo = ln2_split()
    rep = check(c1, c2, gc)
    g32, g32_mid, g32_err = g32_coeffs()
    rep["g32_abs"] = g32_err
    for k, v in rep.items():
        print(f"{k}: {v:.3e}")
    lines = [
        "// sl_smoothing_coeffs.h -- GENERATED by gen_smoothing.py; do not edit.",
        "// Constants of the double-precision smoothing factors s1, s2 (Sec. 3.4).",
        f"// Achieved max errors (double evaluation): series F1 rel {rep['series_rel_F1']:.2e},"
        f" F2 rel {rep['series_rel_F2']:.2e}; g abs {rep['g_abs']:.2e}.",
        "#pragma once",
        "namespace sl {",
        f"constexpr double kSeriesQMax = {SERIES_Q_MAX!r};",
        f"constexpr int kSeriesTerms = {SERIES_TERMS};",
        "// sqrt(pi)^-1 * (-1)^n 8 (n+1)(n+2) / (3 (2n+1) n!): F1(q) = sum kF1[n] q^n",
        "constexpr double kF1[kSeriesTerms] = {" + ", ".join(fmt(c) for c in c1) + "};",
        "// sqrt(pi)^-1 * (-1)^n 16 (n+2)(n+3) / (3 (2n+3) n!): F2(q) = sum kF2[n] q^n",
        "constexpr double kF2[kSeriesTerms] = {" + ", ".join(fmt(c) for c in c2) + "};",
        f"constexpr double kGK = {G_K!r};   // t = kGK / (kGK + p)",
        f"constexpr int kGDeg = {G_DEG};",
        "// g(p) = exp(p^2) erfc(p) ~= sum kG[i] t^i on 0.5 <= p <= 6.9",
        "constexpr double kG[kGDeg + 1] = {" + ", ".join(fmt(c) for c in gc) + "};",
        f"constexpr int kExpDeg = {EXP_DEG};",
        "// Taylor coefficients 1/k! of e^x",
        "constexpr double kExpC[kExpDeg + 1] = {" +
        ", ".join(fmt(mp.mpf(1) / mp.factorial(k)) for k in range(EXP_DEG + 1)) + "};",
        f"constexpr double kLn2Hi = {hi!r};",
        f"constexpr double kLn2Lo = {lo!r};",
        f"constexpr double kLog2E = {float(1 / mp.log(2))!r};",
        f"// single precision (mixed path), 0.5 <= p < 5, g abs error {g32_err:.2e}:",
        f"// g(p) ~= sum kG32[i] (t - kG32Mid)^i, t = kGK / (kGK + p)",
        f"constexpr int kG32Deg = {G32_DEG};",
        f"constexpr float kG32Mid = {g32_mid!r}f;",
        "constexpr float kG32[kG32Deg + 1] = {" + ", ".join(f"{c:.9e}f" for c in g32) + "};",
        "}  // namespace sl",
        "",
    ]
    open(OUT, "w").write("\n".join(lines))
    print("wrote", OUT)


if __name__ == "__main__":
    main()
