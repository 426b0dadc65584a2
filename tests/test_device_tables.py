"""CPU checks of the constant tables that the HIP kernels evaluate, against 40-digit values of
the smoothing factors of Sec. 3.4 (mpmath, independent of both the kernels and the oracle)."""
import math
import struct
import os
import re

import mpmath as mp
import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "paper_2310_13908_amd", "csrc", "sl_smoothing_coeffs.h")


def header():
    return open(HEADER).read()


def int_const(src, name):
    return int(re.search(rf"constexpr int {name} = (\d+);", src).group(1))


def float_const(src, name):
    return float(re.search(rf"constexpr float {name} = ([-+0-9.e]+)f;", src).group(1))


def f1_f2(q):
    """F1 = s1(p)/p and F2 = s2(p)/p^3 at q = p^2 (r = 0 limits at q = 0), 40 digits."""
    mp.mp.dps = 40
    q = mp.mpf(q)
    if q == 0:
        return float(16 / (3 * mp.sqrt(mp.pi))), float(32 / (3 * mp.sqrt(mp.pi)))
    p = mp.sqrt(q)
    e = mp.exp(-q) / mp.sqrt(mp.pi)
    s1 = mp.erf(p) - mp.mpf(2) / 3 * p * (2 * q - 5) * e
    s2 = mp.erf(p) - mp.mpf(2) / 3 * p * (4 * q * q - 14 * q + 3) * e
    return float(s1 / p), float(s2 / p ** 3)


def fma32(a, b, c):
    return np.float32(np.float64(a) * np.float64(b) + np.float64(c))


def test_single_precision_smoothing_table():
    """The mixed path's table of cubics in q reproduces F1 and F2 on 0 <= q < 25 to 3e-7
    relative, evaluated in single precision the way the kernels do (clamped interval index,
    local variable, Horner with fused multiply-adds)."""
    src = header()
    n = int_const(src, "kTab32N")
    qmax = float_const(src, "kTab32QMax")
    assert qmax == 25.0     # p < 5, where s1 = s2 = 1 to single precision
    body = src[src.index("kTab32[2 * kTab32N][4] = {"):]
    rows = re.findall(r"\{([^{}]+)\}", body)[: 2 * n]
    tab = np.array([[float(v.strip().rstrip("f")) for v in r.split(",")] for r in rows], dtype=np.float32)
    assert tab.shape == (2 * n, 4)
    scale = np.float32(n / qmax)
    top = np.float32(n - 2.0 ** -16)
    rng = np.random.default_rng(11)
    qs = np.concatenate([[0.0, 1e-6, 1e-3], np.arange(n) * qmax / n,        # interval starts
                         rng.uniform(0.0, qmax, 400), np.linspace(24.9, qmax * (1 - 1e-7), 5)])
    worst = [0.0, 0.0]
    for q in qs.astype(np.float32):
        u = min(np.float32(q * scale), top)
        i = int(u)
        x = np.float32(u - np.float32(i))
        ref = f1_f2(float(q))
        for k in range(2):
            c = tab[k * n + i]
            v = fma32(fma32(fma32(c[3], x, c[2]), x, c[1]), x, c[0])
            worst[k] = max(worst[k], abs(float(v) - ref[k]) / ref[k])
    assert worst[0] < 3e-7 and worst[1] < 3e-7, worst


def test_table_limits_at_zero():
    """Row 0 starts at the r = 0 limits 16/(3 sqrt(pi)) and 32/(3 sqrt(pi)) of Sec. 3.4."""
    src = header()
    body = src[src.index("kTab32[2 * kTab32N][4] = {"):]
    n = int_const(src, "kTab32N")
    rows = re.findall(r"\{([^{}]+)\}", body)
    c1 = float(rows[0].split(",")[0].strip().rstrip("f"))
    c2 = float(rows[n].split(",")[0].strip().rstrip("f"))
    assert abs(c1 - 16 / (3 * math.sqrt(math.pi))) < 3e-7 * c1
    assert abs(c2 - 32 / (3 * math.sqrt(math.pi))) < 3e-7 * c2


def double_consts(src, name):
    body = re.search(rf"constexpr double {name}\[[^\]]*\] = \{{([^}}]+)\}};", src).group(1)
    return [float(v) for v in body.split(",")]


def double_const(src, name):
    return float(re.search(rf"constexpr double {name} = ([-+0-9.e]+);", src).group(1))


def horner(c, x):
    v = c[-1]
    for a in c[-2::-1]:
        v = v * x + a
    return v


def test_double_precision_smoothing_polynomials():
    """The FP64 kernels' approximations, evaluated as the kernels do, against 40-digit values:
    F1, F2 as polynomials in q - 1/2 on q < 1, and s = 1 - e^{-q} (g(p) + P(p)) on 1 <= p < 6.9
    with g = e^{p^2} erfc(p) fitted in t = 3/(3+p) and e^{-q} = 2^-n e^{-f}."""
    src = header()
    mid, k = double_const(src, "kSeriesMid"), double_const(src, "kGK")
    gmid = double_const(src, "kGMid")
    c1, c2 = double_consts(src, "kF1"), double_consts(src, "kF2")
    g, ec = double_consts(src, "kG"), double_consts(src, "kExpC")
    ln2hi, ln2lo, log2e = double_const(src, "kLn2Hi"), double_const(src, "kLn2Lo"), double_const(src, "kLog2E")
    worst_small = 0.0
    for q in np.concatenate([[0.0], np.linspace(0.0, 1.0, 101)[1:-1], [1.0 - 1e-12]]):
        ref = f1_f2(q)
        worst_small = max(worst_small, abs(horner(c1, q - mid) - ref[0]) / ref[0],
                          abs(horner(c2, q - mid) - ref[1]) / ref[1])
    assert worst_small < 1e-15, worst_small
    c0 = 2.0 / (3.0 * math.sqrt(math.pi))
    worst_large = 0.0
    for p in np.linspace(1.0, 6.9, 150):
        q = p * p
        n = float(np.rint(q * log2e))
        f = (q - n * ln2hi) - n * ln2lo
        E = math.ldexp(horner(ec, -f), -int(n))
        gv = horner(g, k / (k + p) - gmid)
        s1 = 1.0 - E * (gv + c0 * p * (2 * q - 5))
        s2 = 1.0 - E * (gv + c0 * p * (4 * q * q - 14 * q + 3))
        r1, r2 = f1_f2(q)
        worst_large = max(worst_large, abs(s1 / p - r1) / r1, abs(s2 / p ** 3 - r2) / r2)
    assert worst_large < 2e-15, worst_large


def s1_s2(q):
    """s1 and s2 at q = p^2, 40 digits."""
    mp.mp.dps = 40
    q = mp.mpf(q)
    p = mp.sqrt(q)
    e = mp.exp(-q) / mp.sqrt(mp.pi)
    return (float(mp.erf(p) - mp.mpf(2) / 3 * p * (2 * q - 5) * e),
            float(mp.erf(p) - mp.mpf(2) / 3 * p * (4 * q * q - 14 * q + 3) * e))


def test_double_precision_smoothing_table():
    """The FP64 kernels' table: row 0 gives F1, F2 on 0 <= q < 1 to 4e-16 relative, the octave
    rows give s1, s2 on 1 <= q < 48 (past 6.9^2 = 47.61, where s = 1 to double precision) to
    4e-16 absolute (s is of order one there), with the row chosen the way the kernels do (bits 18
    and up of the high word of q: biased exponent and top two mantissa bits) and Horner in double
    precision (two roundings a step here; the kernels fuse them).  Both ends of every row and
    random points are checked; the row choice agrees with frexp's exponent and mantissa; q past
    the table takes the identity row the kernels append, which gives s1 = s2 = 1 exactly."""
    src = header()
    deg = int_const(src, "kTab64Deg")
    n = int_const(src, "kTab64N")
    body = src[src.index("kTab64[kTab64N][kTab64Row] = {"):]
    rows = re.findall(r"\{([^{}]+)\}", body)[:n]
    tab = np.array([[float(v) for v in r.split(",")] for r in rows])
    assert tab.shape == (n, 2 * (deg + 2))
    identity = np.zeros(2 * (deg + 2))
    identity[-2:] = 1.0
    tab = np.vstack([tab, identity])

    def row_of(q):
        hi = struct.unpack("<Q", struct.pack("<d", q))[0] >> 32
        hi = hi - (1 << 32) if hi >= 1 << 31 else hi       # the kernels' int
        return min(max((hi >> 18) - (4 * 1023 - 1), 0), n)

    def row_by_frexp(q):
        if q < 1.0:
            return 0
        m, e = math.frexp(q)                # q = m 2^e, 0.5 <= m < 1
        return min(1 + 4 * (e - 1) + int((m - 0.5) * 8.0), n)

    def evaluate(q):
        r = tab[row_of(q)]
        x = (q - r[0]) * r[1]
        p1, p2 = r[2], r[3]
        for k in range(1, deg + 1):
            p1 = p1 * x + r[2 + 2 * k]
            p2 = p2 * x + r[3 + 2 * k]
        return p1, p2

    qend = 48.0
    edges = [0.0, 1.0] + [2.0 ** e * (1 + j / 4) for e in range(6) for j in range(4)]
    qs = [q for q in edges if q < qend] + [math.nextafter(q, 0.0) for q in edges[1:] if q <= qend]
    qs += list(np.random.default_rng(5).uniform(0.0, qend, 300)) + [1e-9, 0.5, 6.9 ** 2]
    worst = 0.0
    for q in qs:
        assert row_of(q) == row_by_frexp(q), q
        p1, p2 = evaluate(q)
        if q < 1.0:
            e1, e2 = f1_f2(q)
            worst = max(worst, abs(p1 - e1) / e1, abs(p2 - e2) / e2)
        else:
            e1, e2 = s1_s2(q)
            worst = max(worst, abs(p1 - e1), abs(p2 - e2))
    assert worst < 4e-16, worst
    assert row_of(math.nextafter(qend, 0.0)) == n - 1 and row_of(-0.0) == 0
    for q in (qend, 60.0, 1e300, math.inf, math.nan):
        assert row_of(q) == n
    for q in (qend, 60.0, 1e300):
        assert evaluate(q) == (1.0, 1.0)
