#!/usr/bin/env python3
"""Generate sl_smoothing_coeffs.h: constants of the device evaluation of the smoothing factors
s1, s2 of Sec. 3.4 (s1(p) = erf p - (2/3) p (2p^2 - 5) e^{-p^2}/sqrt(pi),
s2(p) = erf p - (2/3) p (4p^4 - 14p^2 + 3) e^{-p^2}/sqrt(pi)).

The device code splits the regularized zone p = r/delta < 6.9 in two:

* q = p^2 < 1: F1 = s1(p)/p and F2 = s2(p)/p^3 as polynomials in x = q - 1/2, the interpolants
  at Chebyshev nodes of [0, 1] of 40-digit values.  Both are entire functions of q with the
  r -> 0 limits F1(0) = 16/(3 sqrt(pi)), F2(0) = 32/(3 sqrt(pi)) of Sec. 3.4, and the
  polynomial has no cancellation near q = 0, where s2 itself loses all its digits.
* 1 <= p < 6.9: s = 1 - e^{-q} (g(p) + P(p)) with the exact polynomial parts
  P1 = (2/3)p(2q-5)/sqrt(pi), P2 = (2/3)p(4q^2-14q+3)/sqrt(pi) and the scaled complementary
  error function g(p) = e^{p^2} erfc(p).  g enters s only through e^{-q} g, so its polynomial
  (in t - t_mid, t = 3/(3+p)) is a least-squares fit weighted by e^{-q}: the weighted error
  e^{-q} |g_fit - g| is what perturbs s.  e^{-q} = 2^-n e^{-f}, n = rint(q / ln 2),
  |f| <= ln2/2, with e^x on |x| <= ln2/2 interpolated at Chebyshev nodes.

The mixed-precision path evaluates F1 and F2 in single precision from a table of cubics in q:
0 <= q < 25 is cut into TAB32_N equal intervals, and on interval i, with the local variable
x = q TAB32_N / 25 - i in [0, 1), F = c0 + x (c1 + x (c2 + x c3)), the interpolant at the four
Chebyshev nodes of the interval of 40-digit values, rounded to single precision.  K1 = F1/delta
and K2 = F2/delta^3 then take one table row, three fused multiply-adds per factor and no
transcendental instruction; there is no cancellation anywhere in q.

The double-precision kernels evaluate the whole zone q < 6.9^2 from one table of polynomials of
degree TAB64_DEG: interval 0 is 0 <= q < 1, where F1 and F2 are taken (as above, entire in q);
interval 1 + 4 e + j covers q in 2^e [1 + j/4, 1 + (j+1)/4), e = 0..5, j = 0..3, where s1 and s2
themselves are taken (they stay away from their branch point at q = 0 there).  On each interval,
with centre m and half width h, the polynomial in x = (q - m)/h in [-1, 1] interpolates 40-digit
values at Chebyshev nodes; K1 = F1/delta or s1/r, K2 = F2/delta^3 or s2/r^3.  One branch and one
table row per pair, instead of a series for q < 1 and an exp/erfc form beyond.

Run: python gen_smoothing.py  (rewrites sl_smoothing_coeffs.h next to this file and prints the
achieved double-precision error of every approximation).
"""
from __future__ import annotations

import os
import struct

import mpmath as mp
import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
OUT = os.path.join(HERE, "sl_smoothing_coeffs.h")

SERIES_Q_MAX = 1.0      # small-q polynomial used for q = p^2 below this
SERIES_MID = 0.5        # ... in x = q - SERIES_MID
SERIES_DEG = 12
G_LO, G_HI = 1.0, 6.9   # range of the g fit (p)
G_K = 3.0               # t = G_K / (G_K + p)
G_DEG = 11
EXP_DEG = 11            # degree of e^x on |x| <= ln2/2
# Single-precision smoothing of the mixed path: cubics on TAB32_N equal intervals of
# 0 <= q < TAB32_QMAX (p < 5, where s = 1 to single precision).
TAB32_N = 256
TAB32_QMAX = 25.0
# Double precision: degree and intervals of the table (see above).
TAB64_DEG = 13
TAB64_QMAX = 6.9 ** 2


def cheb_nodes(a, b, n):
    return [(a + b) / 2 + (b - a) / 2 * mp.cos(mp.pi * (j + mp.mpf(1) / 2) / n) for j in range(n)]


def F_exact(q):
    q = mp.mpf(q)
    sp = mp.sqrt(mp.pi)
    if q == 0:
        return 16 / (3 * sp), 32 / (3 * sp)
    s1, s2 = s_exact(mp.sqrt(q))
    p = mp.sqrt(q)
    return s1 / p, s2 / p ** 3


def series_coeffs():
    """Interpolants of F1, F2 at Chebyshev nodes of [0, SERIES_Q_MAX], in x = q - SERIES_MID."""
    xs = cheb_nodes(mp.mpf(0), mp.mpf(SERIES_Q_MAX), SERIES_DEG + 1)
    A = mp.matrix([[(x - SERIES_MID) ** i for i in range(SERIES_DEG + 1)] for x in xs])
    vals = [F_exact(x) for x in xs]
    c1 = mp.lu_solve(A, mp.matrix([v[0] for v in vals]))
    c2 = mp.lu_solve(A, mp.matrix([v[1] for v in vals]))
    return [c for c in c1], [c for c in c2]


def g_exact(p):
    p = mp.mpf(p)
    return mp.exp(p * p) * mp.erfc(p)


def g_tmid():
    return float((G_K / (G_K + G_HI) + G_K / (G_K + G_LO)) / 2)


def g_coeffs():
    """Least squares (40-digit normal equations) of g in t - t_mid, weighted by e^{-p^2}."""
    mid = mp.mpf(g_tmid())
    ps = [mp.mpf(G_LO) + (G_HI - G_LO) * (1 - mp.cos(mp.pi * (k + mp.mpf(1) / 2) / 600)) / 2
          for k in range(600)]
    rows, rhs = [], []
    for p in ps:
        w = mp.exp(-p * p)
        t = G_K / (G_K + p) - mid
        rows.append([w * t ** i for i in range(G_DEG + 1)])
        rhs.append(w * g_exact(p))
    A = mp.matrix(rows)
    y = mp.matrix(rhs)
    return [c for c in mp.lu_solve(A.T * A, A.T * y)]


def exp_coeffs():
    """Interpolant of e^x at Chebyshev nodes of [-ln2/2, ln2/2] (monomial coefficients)."""
    a = mp.log(2) / 2
    xs = cheb_nodes(-a, a, EXP_DEG + 1)
    A = mp.matrix([[x ** i for i in range(EXP_DEG + 1)] for x in xs])
    return [c for c in mp.lu_solve(A, mp.matrix([mp.exp(x) for x in xs]))]


def tab32_coeffs():
    """Per interval, the cubic in x in [0, 1) through F1, F2 at the interval's Chebyshev nodes."""
    nodes = [(1 + mp.cos(mp.pi * (j + mp.mpf(1) / 2) / 4)) / 2 for j in range(4)]
    A = mp.matrix([[x ** i for i in range(4)] for x in nodes])
    h = mp.mpf(TAB32_QMAX) / TAB32_N
    t1, t2 = [], []
    for i in range(TAB32_N):
        vals = [F_exact(h * (i + x)) for x in nodes]
        c1 = mp.lu_solve(A, mp.matrix([v[0] for v in vals]))
        c2 = mp.lu_solve(A, mp.matrix([v[1] for v in vals]))
        t1.append([float(np.float32(float(c))) for c in c1])
        t2.append([float(np.float32(float(c))) for c in c2])
    return t1, t2


def tab64_intervals():
    iv = [(0.0, 1.0)]
    for e in range(6):
        for j in range(4):
            a, b = 2.0 ** e * (1 + j / 4), 2.0 ** e * (1 + (j + 1) / 4)
            if a < TAB64_QMAX:
                iv.append((a, b))
    return iv


def S_exact(q):
    return s_exact(mp.sqrt(mp.mpf(q)))


def tab64_rows():
    """Per interval: centre, 1/half width, then (c1_k, c2_k) for k = TAB64_DEG .. 0 (Horner order)."""
    n = TAB64_DEG + 1
    xs = [mp.cos(mp.pi * (j + mp.mpf(1) / 2) / n) for j in range(n)]
    A = mp.matrix([[x ** i for i in range(n)] for x in xs])
    rows = []
    for idx, (a, b) in enumerate(tab64_intervals()):
        f = F_exact if idx == 0 else S_exact
        m, h = (mp.mpf(a) + mp.mpf(b)) / 2, (mp.mpf(b) - mp.mpf(a)) / 2
        vals = [f(m + h * x) for x in xs]
        c1 = mp.lu_solve(A, mp.matrix([v[0] for v in vals]))
        c2 = mp.lu_solve(A, mp.matrix([v[1] for v in vals]))
        row = [float(m), float(1 / h)]
        for k in range(TAB64_DEG, -1, -1):
            row += [float(c1[k]), float(c2[k])]
        rows.append(row)
    return rows


def tab64_error(rows):
    """Worst relative error of F (interval 0) and absolute error of s (the others), double
    evaluation with two roundings per Horner step (the device fuses them)."""
    worst = 0.0
    for idx, (a, b) in enumerate(tab64_intervals()):
        f = F_exact if idx == 0 else S_exact
        r = rows[idx]
        for q in np.linspace(a, min(b, TAB64_QMAX), 40):
            x = (q - r[0]) * r[1]
            p1, p2 = r[2], r[3]
            for k in range(1, TAB64_DEG + 1):
                p1 = p1 * x + r[2 + 2 * k]
                p2 = p2 * x + r[3 + 2 * k]
            e1, e2 = (float(v) for v in f(q))
            d1, d2 = abs(p1 - e1), abs(p2 - e2)
            if idx == 0:
                d1, d2 = d1 / abs(e1), d2 / abs(e2)
            worst = max(worst, d1, d2)
    return worst


def tab32_error(t1, t2):
    """Max relative error of F1, F2 from the table, evaluated in single precision as on the
    device (q rounded to single precision first; the error of that rounding is not counted)."""
    f32 = np.float32
    scale = f32(TAB32_N / TAB32_QMAX)
    rng = np.random.default_rng(7)
    qs = np.concatenate([np.linspace(0.0, TAB32_QMAX, 1201)[:-1],
                         rng.uniform(0.0, TAB32_QMAX, 800)]).astype(np.float32)
    worst = [0.0, 0.0]
    for q in qs:
        u = min(f32(q * scale), f32(np.nextafter(f32(TAB32_N), f32(0))))
        i = int(u)
        x = f32(u - f32(i))
        ex = F_exact(float(q))
        for k, tab in enumerate((t1, t2)):
            c = [f32(v) for v in tab[i]]
            v = f32(f32(f32(f32(f32(c[3] * x) + c[2]) * x) + c[1]) * x + c[0])
            worst[k] = max(worst[k], float(abs(mp.mpf(float(v)) - ex[k]) / ex[k]))
    return worst


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


def check(c1, c2, gc, ec):
    """Max errors of the double-precision evaluation (numpy mirrors the device arithmetic)."""
    rep = {}
    q = np.linspace(0.0, SERIES_Q_MAX, 2001)
    F1 = horner(c1, q - SERIES_MID)
    F2 = horner(c2, q - SERIES_MID)
    e1 = e2 = 0.0
    for qi, a, b in zip(q[::5], F1[::5], F2[::5]):
        r1, r2 = F_exact(float(qi))
        e1 = max(e1, float(abs(a - r1) / r1))
        e2 = max(e2, float(abs(b - r2) / r2))
    rep["series_rel_F1"], rep["series_rel_F2"] = e1, e2
    p = np.linspace(G_LO, G_HI, 3001)
    gv = horner(gc, G_K / (G_K + p) - g_tmid())
    rep["g_weighted_abs"] = max(float(abs(mp.mpf(float(a)) - g_exact(float(x))) * mp.exp(-mp.mpf(float(x)) ** 2))
                                for x, a in zip(p[::3], gv[::3]))
    a = float(mp.log(2) / 2)
    x = np.linspace(-a, a, 2001)
    ev = horner(ec, x)
    rep["exp_rel"] = max(float(abs(mp.mpf(float(v)) - mp.exp(float(xx))) / mp.exp(float(xx)))
                         for xx, v in zip(x[::5], ev[::5]))
    # the assembled smoothing factors on 1 <= p < 6.9 (double evaluation, exact e^{-q})
    worst = 0.0
    c0 = 2.0 / (3.0 * np.sqrt(np.pi))
    for pp in np.linspace(G_LO, G_HI, 400):
        qq = pp * pp
        g = horner(gc, np.array([G_K / (G_K + pp) - g_tmid()]))[0]
        E = float(mp.exp(-mp.mpf(qq)))
        s1 = 1.0 - E * (g + c0 * pp * (2 * qq - 5))
        s2 = 1.0 - E * (g + c0 * pp * (4 * qq * qq - 14 * qq + 3))
        x1, x2 = s_exact(pp)
        worst = max(worst, float(abs(s1 - x1) / x1), float(abs(s2 - x2) / x2))
    rep["s_rel_1_to_6.9"] = worst
    return rep


def fmt(v):
    return f"{float(v):.17e}"


def main():
    mp.mp.dps = 40
    c1, c2 = series_coeffs()
    gc = g_coeffs()
    ec = exp_coeffs()
    hi, lo = ln2_split()
    rep = check(c1, c2, gc, ec)
    t1, t2 = tab32_coeffs()
    rep["tab32_rel_F1"], rep["tab32_rel_F2"] = tab32_error(t1, t2)
    r64 = tab64_rows()
    rep["tab64_err"] = tab64_error(r64)
    for k, v in rep.items():
        print(f"{k}: {v:.3e}")
    lines = [
        "// sl_smoothing_coeffs.h -- GENERATED by gen_smoothing.py; do not edit.",
        "// Constants of the device evaluation of the smoothing factors s1, s2 (Sec. 3.4).",
        f"// Achieved max errors (double evaluation): F1 rel {rep['series_rel_F1']:.2e},"
        f" F2 rel {rep['series_rel_F2']:.2e}; e^-q |g - fit| {rep['g_weighted_abs']:.2e};"
        f" exp rel {rep['exp_rel']:.2e}; s on [1, 6.9) rel {rep['s_rel_1_to_6.9']:.2e}.",
        "#pragma once",
        "namespace sl {",
        f"constexpr double kSeriesQMax = {SERIES_Q_MAX!r};",
        f"constexpr double kSeriesMid = {SERIES_MID!r};",
        f"constexpr int kSeriesDeg = {SERIES_DEG};",
        "// F1(q) = s1(p)/p ~= sum kF1[n] (q - kSeriesMid)^n on 0 <= q < kSeriesQMax",
        "constexpr double kF1[kSeriesDeg + 1] = {" + ", ".join(fmt(c) for c in c1) + "};",
        "// F2(q) = s2(p)/p^3 ~= sum kF2[n] (q - kSeriesMid)^n on 0 <= q < kSeriesQMax",
        "constexpr double kF2[kSeriesDeg + 1] = {" + ", ".join(fmt(c) for c in c2) + "};",
        f"constexpr double kGK = {G_K!r};   // t = kGK / (kGK + p)",
        f"constexpr double kGMid = {g_tmid()!r};",
        f"constexpr int kGDeg = {G_DEG};",
        f"// g(p) = exp(p^2) erfc(p) ~= sum kG[i] (t - kGMid)^i on {G_LO} <= p <= {G_HI}",
        "constexpr double kG[kGDeg + 1] = {" + ", ".join(fmt(c) for c in gc) + "};",
        f"constexpr int kExpDeg = {EXP_DEG};",
        "// e^x ~= sum kExpC[k] x^k on |x| <= ln2/2",
        "constexpr double kExpC[kExpDeg + 1] = {" + ", ".join(fmt(c) for c in ec) + "};",
        f"constexpr double kLn2Hi = {hi!r};",
        f"constexpr double kLn2Lo = {lo!r};",
        f"constexpr double kLog2E = {float(1 / mp.log(2))!r};",
        "// Single precision (mixed path), 0 <= q < kTab32QMax: interval i = floor(x'), x' = q kTab32N /",
        "// kTab32QMax, x = x' - i; F1 ~= c0 + x (c1 + x (c2 + x c3)) with c = kTab32[i][0..3], F2 likewise",
        f"// from kTab32[kTab32N + i].  Max relative error F1 {rep['tab32_rel_F1']:.2e}, F2 {rep['tab32_rel_F2']:.2e}.",
        f"constexpr int kTab32N = {TAB32_N};",
        f"constexpr float kTab32QMax = {TAB32_QMAX!r}f;",
        "constexpr float kTab32[2 * kTab32N][4] = {",
        *["    {" + ", ".join(f"{c:.9e}f" for c in row) + "}," for row in t1 + t2],
        "};",
        "// Double precision, 0 <= q < 6.9^2: row i = {centre, 1/half width, (c1, c2) of x^kTab64Deg, ...,",
        "// (c1, c2) of x^0}, x = (q - centre)/half width; row 0: F1, F2 on [0, 1); row 1 + 4 e + j: s1, s2 on",
        f"// 2^e [1 + j/4, 1 + (j+1)/4).  Max error (relative for F, absolute for s) {rep['tab64_err']:.2e}.",
        f"constexpr int kTab64Deg = {TAB64_DEG};",
        f"constexpr int kTab64N = {len(r64)};",
        "constexpr int kTab64Row = 2 * (kTab64Deg + 2);   // doubles per row",
        "constexpr double kTab64[kTab64N][kTab64Row] = {",
        *["    {" + ", ".join(f"{c:.17e}" for c in row) + "}," for row in r64],
        "};",
        "}  // namespace sl",
        "",
    ]
    open(OUT, "w").write("\n".join(lines))
    print("wrote", OUT)


if __name__ == "__main__":
    main()
