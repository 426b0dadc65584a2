// sl_device.h -- device arithmetic of the regularized Stokes single layer on gfx950.
//
// Pair term (Sec. 3.4, eq. (regstokes)), for target t, source x with packed density
// g = w f (the trapezoid-POU weight of Sec. 3.3 folded into the force), d = t - x, r = |d|:
//
//     term = K1 g + K2 (g . d) d,   K1 = s1(r/delta)/r,  K2 = s2(r/delta)/r^3.
//
// Far from the target (r/delta >= 6.9) both smoothing factors equal 1 to double precision
// (|s - 1| < 2^-53; at r/delta >= 5, |s - 1| < 2^-24), so the far pair is the plain
// Stokeslet K1 = 1/r, K2 = 1/r^3: 28 flops, no erf/exp.  Nearer pairs apply the smoothing in
// double precision (below: a fitted polynomial in (r/delta)^2 for r < delta, otherwise one exp
// and a fitted scaled complementary error function).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "sl_smoothing_coeffs.h"

namespace sl {

constexpr int kWave = 64;            // CDNA wavefront width
constexpr int kCluster = 64;         // sources per cluster (one classification unit)
constexpr int kPad = 256;            // point arrays are padded to a multiple of this
constexpr double kC0 = 0.376126389031837524632052967707181724;   // 2 / (3 sqrt(pi))
constexpr double kRhoExact64 = 6.9;  // s1 = s2 = 1 in double precision beyond this r/delta
constexpr double kRhoExact32 = 5.0;  // ... and in single precision beyond this r/delta
constexpr double kRho64Min = 0.0;    // smallest double-precision zone of the mixed path: none
                                     // (the single-precision smoothing table spans 0 <= p < 5)

// 1/sqrt(x) for finite x > 0 to ~1 ulp: hardware estimate (good to about 2^-23 relative)
// refined by one third-order step y (1 + e/2 + 3e^2/8), e = 1 - x y^2.
__device__ __forceinline__ double rsqrt64(double x)
{
    const double y = __builtin_amdgcn_rsq(x);
    const double t = x * y;
    const double e = fma(-t, y, 1.0);
    const double p = fma(e, 0.375, 0.5);
    return fma(y * e, p, y);
}

// Plain Stokeslet pair in double precision, accumulated into (ax, ay, az).
__device__ __forceinline__ void far_pair64(double tx, double ty, double tz,
                                           double sx, double sy, double sz,
                                           double gx, double gy, double gz,
                                           double &ax, double &ay, double &az)
{
    const double dx = tx - sx, dy = ty - sy, dz = tz - sz;
    const double r2 = fma(dx, dx, fma(dy, dy, dz * dz));
    const double ri = rsqrt64(r2);
    const double ri2 = ri * ri;
    const double gd = fma(gx, dx, fma(gy, dy, gz * dz));
    const double c = gd * ri2;
    ax = fma(ri, fma(c, dx, gx), ax);
    ay = fma(ri, fma(c, dy, gy), ay);
    az = fma(ri, fma(c, dz, gz), az);
}

// Per-target constants of the smoothing: powers of 1/delta and the squared radius inside
// which the smoothing differs from 1 in double precision.
struct DeltaC {
    double id, id2, id3, cut2;
};

__device__ __forceinline__ DeltaC make_delta(double delta)
{
    DeltaC c;
    c.id = 1.0 / delta;
    c.id2 = c.id * c.id;
    c.id3 = c.id2 * c.id;
    const double rc = kRhoExact64 * delta;
    c.cut2 = rc * rc;
    return c;
}

// A polynomial coefficient placed in a scalar register where it is used.  Without this the
// compiler hoists the ~60 double constants of the smoothing out of the source loop into vector
// registers, which costs more than a hundred VGPRs and halves the occupancy; rematerializing
// them with scalar moves keeps them off the vector register file.
__device__ __forceinline__ double sconst(double c)
{
    asm volatile("" : "+s"(c));
    return c;
}

// e^{-q} for 0 <= q <= 700: q = n ln2 + f with |f| <= ln2/2, e^{-q} = 2^-n e^{-f}, e^{-f} by
// a degree-11 polynomial fitted on |f| <= ln2/2 (relative error below 2^-52).
__device__ __forceinline__ double exp_neg64(double q)
{
    const double n = rint(q * kLog2E);
    const double f = fma(-n, kLn2Lo, fma(-n, kLn2Hi, q));
    double p = kExpC[kExpDeg];
#pragma unroll
    for (int k = kExpDeg - 1; k >= 0; --k) p = fma(p, -f, sconst(kExpC[k]));
    return ldexp(p, -(int)n);
}

// Smoothed kernel factors for q = (r/delta)^2 < 1 (Sec. 3.4): K1 = F1(q)/delta,
// K2 = F2(q)/delta^3 with F1 = s1(p)/p, F2 = s2(p)/p^3 as polynomials in q - 1/2.  No 1/r is
// needed, there is no cancellation, and the r = 0 limits 16/(3 sqrt(pi) delta),
// 32/(3 sqrt(pi) delta^3) come out at q = 0.
__device__ __forceinline__ void smoothing_small64(double q, const DeltaC &dc, double &K1, double &K2)
{
    const double x = q - kSeriesMid;
    double f1 = kF1[kSeriesDeg], f2 = kF2[kSeriesDeg];
#pragma unroll
    for (int k = kSeriesDeg - 1; k >= 0; --k) {
        f1 = fma(f1, x, sconst(kF1[k]));
        f2 = fma(f2, x, sconst(kF2[k]));
    }
    K1 = f1 * dc.id;
    K2 = f2 * dc.id3;
}

// Smoothed kernel factors for 1 <= q, p = r/delta < 6.9, given r2 = r^2 and ri = 1/r:
// s = 1 - e^{-q} (g(p) + P(p)), g(p) = e^{p^2} erfc(p) from its fitted polynomial in
// t = 3/(3+p), P1 = (2/(3 sqrt(pi))) p (2q - 5), P2 = (2/(3 sqrt(pi))) p (4q^2 - 14q + 3);
// K1 = s1/r, K2 = s2/r^3.
__device__ __forceinline__ void smoothing_large64(double r2, double q, double ri, double ri2,
                                                  const DeltaC &dc, double &K1, double &K2)
{
    const double p = (r2 * ri) * dc.id;
    const double E = exp_neg64(q);
    const double den = kGK + p;
    double y = __builtin_amdgcn_rcp(den);      // refined twice: 1/den to ~1 ulp
    double e = fma(-den, y, 1.0);
    y = fma(y, e, y);
    e = fma(-den, y, 1.0);
    y = fma(y, e, y);
    const double t = fma(kGK, y, -kGMid);
    double g = kG[kGDeg];
#pragma unroll
    for (int i = kGDeg - 1; i >= 0; --i) g = fma(g, t, sconst(kG[i]));
    const double c0p = kC0 * p;
    const double A1 = fma(c0p, fma(2.0, q, -5.0), g);
    const double A2 = fma(c0p, fma(q, fma(4.0, q, -14.0), 3.0), g);
    K1 = ri * fma(-E, A1, 1.0);
    K2 = (ri * ri2) * fma(-E, A2, 1.0);
}

// Regularized pair in double precision: the exact kernel for any r >= 0.
__device__ __forceinline__ void near_pair64(double tx, double ty, double tz,
                                            double sx, double sy, double sz,
                                            double gx, double gy, double gz,
                                            const DeltaC &dc,
                                            double &ax, double &ay, double &az)
{
    const double dx = tx - sx, dy = ty - sy, dz = tz - sz;
    const double r2 = fma(dx, dx, fma(dy, dy, dz * dz));
    const double ri = rsqrt64(r2 > 0.0 ? r2 : 1.0);
    const double ri2 = ri * ri;
    double K1 = ri, K2 = ri * ri2;
    if (r2 < dc.cut2) {
        const double q = r2 * dc.id2;
        if (q < kSeriesQMax) smoothing_small64(q, dc, K1, K2);
        else smoothing_large64(r2, q, ri, ri2, dc, K1, K2);
    }
    const double gd = fma(gx, dx, fma(gy, dy, gz * dz));
    const double c = gd * K2;
    ax = fma(K1, gx, fma(c, dx, ax));
    ay = fma(K1, gy, fma(c, dy, ay));
    az = fma(K1, gz, fma(c, dz, az));
}

// The double-precision smoothing table (kTab64) in LDS, copied by the threads of a workgroup (the
// caller synchronizes afterwards): per row, {centre, 1/half width}, then the pairs (c1, c2) from
// the highest power down, as double2.  Row kTab64N, past the table, is the identity: local
// variable 0 and constant term 1, so that it gives s1 = s2 = 1 exactly.
constexpr int kTab64Row2 = kTab64Row / 2;
constexpr int kTab64Size2 = (kTab64N + 1) * kTab64Row2;

__device__ __forceinline__ void load_tab64(double2 *tab)
{
    for (int i = threadIdx.x; i < kTab64Size2; i += blockDim.x) {
        const int row = i / kTab64Row2, k = i % kTab64Row2;
        tab[i] = row < kTab64N ? make_double2(kTab64[row][2 * k], kTab64[row][2 * k + 1])
                               : (k == kTab64Row2 - 1 ? make_double2(1.0, 1.0)
                                                      : make_double2(0.0, 0.0));
    }
}

// Table row of q = (r/delta)^2 >= 0 from the high word of its bits, whose bits 18 and up hold
// the biased exponent and the top two mantissa bits: 0 for q < 1, 1 + 4 e + j for q in
// 2^e [1 + j/4, 1 + (j+1)/4), and the identity row kTab64N past the table (q >= 48, infinity
// and NaN included).
__device__ __forceinline__ int tab64_row(double q)
{
    const int i = (__double2hiint(q) >> 18) - (4 * 1023 - 1);
    return min(max(i, 0), kTab64N);
}

// Row 0: F1(q) = s1/p and F2(q) = s2/p^3; other rows: s1 and s2; a polynomial of degree
// kTab64Deg in the row's local variable, Horner with fused multiply-adds.
__device__ __forceinline__ void smoothing64(double q, const double2 *tab, int row, double &p1, double &p2)
{
    const double2 *r = tab + row * kTab64Row2;
    const double2 h = r[0];
    const double x = (q - h.x) * h.y;
    double2 c = r[1];
    p1 = c.x;
    p2 = c.y;
#pragma unroll
    for (int k = 2; k < kTab64Row2; ++k) {
        c = r[k];
        p1 = fma(p1, x, c.x);
        p2 = fma(p2, x, c.y);
    }
}

// One source against the R targets of a lane, in double precision, the smoothing from the table
// in LDS (`tab`, load_tab64), evaluated wherever one lane of the wavefront is within 6.9 delta:
// one branch, one table row a pair.  Lanes past the table take its identity row, which leaves
// the plain kernel unchanged, and lanes between 6.9 delta and the table's end (s = 1 to double
// precision there) take s from the table.
template <int R>
__device__ __forceinline__ void near_pairs64(const double (&tx)[R], const double (&ty)[R],
                                             const double (&tz)[R], double sx, double sy, double sz,
                                             double gx, double gy, double gz, const DeltaC (&dc)[R],
                                             const double2 *tab, double (&ax)[R], double (&ay)[R],
                                             double (&az)[R])
{
    double dx[R], dy[R], dz[R], r2[R], q[R], K1[R], K2[R];
    bool any = false;
#pragma unroll
    for (int r = 0; r < R; ++r) {
        dx[r] = tx[r] - sx;
        dy[r] = ty[r] - sy;
        dz[r] = tz[r] - sz;
        r2[r] = fma(dx[r], dx[r], fma(dy[r], dy[r], dz[r] * dz[r]));
        K1[r] = rsqrt64(r2[r] > 0.0 ? r2[r] : 1.0);
        K2[r] = K1[r] * K1[r] * K1[r];
        q[r] = r2[r] * dc[r].id2;
        any = any || r2[r] < dc[r].cut2;
    }
    if (__builtin_amdgcn_ballot_w64(any)) {
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int row = tab64_row(q[r]);
            double p1, p2;
            smoothing64(q[r], tab, row, p1, p2);
            // row 0 holds F1 = s1/p and F2 = s2/p^3 (finite at r = 0), the others s1 and s2
            const bool inner = row == 0;
            K1[r] = (inner ? dc[r].id : K1[r]) * p1;
            K2[r] = (inner ? dc[r].id3 : K2[r]) * p2;
        }
    }
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const double gd = fma(gx, dx[r], fma(gy, dy[r], gz * dz[r]));
        const double c = gd * K2[r];
        ax[r] = fma(K1[r], gx, fma(c, dx[r], ax[r]));
        ay[r] = fma(K1[r], gy, fma(c, dy[r], ay[r]));
        az[r] = fma(K1[r], gz, fma(c, dz[r], az[r]));
    }
}

// Pair of the mixed path's double-precision zone (p < rho64, including r = 0): as near_pair64,
// without 1/r where q < 1 (always so for rho64 <= 1).
__device__ __forceinline__ void zone_pair64(double tx, double ty, double tz,
                                            double sx, double sy, double sz,
                                            double gx, double gy, double gz,
                                            const DeltaC &dc,
                                            double &ax, double &ay, double &az)
{
    const double dx = tx - sx, dy = ty - sy, dz = tz - sz;
    const double r2 = fma(dx, dx, fma(dy, dy, dz * dz));
    const double q = r2 * dc.id2;
    double K1, K2;
    if (q < kSeriesQMax) {
        smoothing_small64(q, dc, K1, K2);
    } else {
        const double ri = rsqrt64(r2);
        const double ri2 = ri * ri;
        K1 = ri;
        K2 = ri * ri2;
        if (r2 < dc.cut2) smoothing_large64(r2, q, ri, ri2, dc, K1, K2);
    }
    const double gd = fma(gx, dx, fma(gy, dy, gz * dz));
    const double c = gd * K2;
    ax = fma(K1, gx, fma(c, dx, ax));
    ay = fma(K1, gy, fma(c, dy, ay));
    az = fma(K1, gz, fma(c, dz, az));
}

// Single-precision constants of the mixed path's near zone for one target: 1/delta, 1/delta^3,
// the table scale kTab32N / (kTab32QMax delta^2) (table position of r^2), and the squared radii
// of its double-precision zone (rho64 delta)^2 and of the smoothing (5 delta)^2.
struct DeltaC32 {
    float id, id3, tsc, cut2_64, cut2_5;
};

__device__ __forceinline__ DeltaC32 make_delta32(double delta, double rho64)
{
    DeltaC32 c;
    c.id = (float)(1.0 / delta);
    c.id3 = (float)(1.0 / (delta * delta * delta));
    c.tsc = (float)((double)kTab32N / ((double)kTab32QMax * delta * delta));
    c.cut2_64 = (float)(rho64 * rho64 * delta * delta);
    c.cut2_5 = (float)(kRhoExact32 * kRhoExact32 * delta * delta);
    return c;
}

// The single-precision smoothing table (F1 rows, then F2 rows; four cubic coefficients a row),
// copied into LDS by the threads of a workgroup.  The caller synchronizes afterwards.
constexpr int kTab32Rows = 2 * kTab32N;

__device__ __forceinline__ void load_tab32(float4 *tab)
{
    for (int i = threadIdx.x; i < kTab32Rows; i += blockDim.x)
        tab[i] = make_float4(kTab32[i][0], kTab32[i][1], kTab32[i][2], kTab32[i][3]);
}

// Smoothed K1 = s1(p)/r = F1(q)/delta and K2 = s2(p)/r^3 = F2(q)/delta^3 in single precision,
// q = (r/delta)^2 < 25, from the table of cubics (no transcendental instruction, no cancellation).
// Positions beyond the table are clamped to its last interval; the caller selects those lanes out.
__device__ __forceinline__ void smoothing32(float r2, const DeltaC32 &dc, const float4 *tab,
                                            float &K1, float &K2)
{
    const float u = fminf(r2 * dc.tsc, (float)kTab32N - 0x1p-16f);
    const int i = (int)u;                          // u >= 0: the floor
    const float x = __builtin_amdgcn_fractf(u);    // u - floor(u), exact here
    const float4 a = tab[i];
    const float4 b = tab[kTab32N + i];
    K1 = fmaf(fmaf(fmaf(a.w, x, a.z), x, a.y), x, a.x) * dc.id;
    K2 = fmaf(fmaf(fmaf(b.w, x, b.z), x, b.y), x, b.x) * dc.id3;
}

// Difference and squared distance in single precision for the mixed path.  Every kernel takes
// them from here, so a pair falls in the same zone (double-precision zone, smoothing, plain) in
// every kernel that looks at it.
__device__ __forceinline__ float diff32(float tx, float ty, float tz, float sx, float sy, float sz,
                                        float &dx, float &dy, float &dz)
{
    dx = tx - sx;
    dy = ty - sy;
    dz = tz - sz;
    return fmaf(dx, dx, fmaf(dy, dy, dz * dz));
}

// Near pair of the mixed path, single-precision zones: rho64 <= p < 5 smoothed, p >= 5 plain,
// accumulated in (px, py, pz); with ZONE, p < rho64 (including r = 0) contributes nothing here --
// the caller sums that zone in double precision (zone_pair64), deciding it with the same diff32
// test.  Without it (rho64 = 0) every pair is summed here, r = 0 through the table's q = 0 row.  The
// smoothing runs only when some lane of the wavefront needs it (a wave-uniform test), so a
// source that is farther than 5 delta from all 64 targets of the wavefront costs what a far pair
// costs.  `tab` is the single-precision smoothing table (load_tab32).
template <bool ZONE = true>
__device__ __forceinline__ void near_pair32(float tx32, float ty32, float tz32, float sx32,
                                            float sy32, float sz32, float gx32, float gy32,
                                            float gz32, const DeltaC32 &dc32, const float4 *tab,
                                            float &px, float &py, float &pz)
{
    float dx, dy, dz;
    const float r2 = diff32(tx32, ty32, tz32, sx32, sy32, sz32, dx, dy, dz);
    const bool z64 = ZONE && r2 < dc32.cut2_64;
    const bool z5 = r2 < dc32.cut2_5;
    const float ri = __builtin_amdgcn_rsqf(r2);
    float K1 = ri, K2 = ri * ri * ri;
    if (__builtin_amdgcn_ballot_w64(z5)) {
        float S1, S2;
        smoothing32(r2, dc32, tab, S1, S2);
        K1 = z5 ? S1 : K1;
        K2 = z5 ? S2 : K2;
    }
    K1 = z64 ? 0.0f : K1;
    K2 = z64 ? 0.0f : K2;
    const float gd = fmaf(gx32, dx, fmaf(gy32, dy, gz32 * dz));
    const float c = gd * K2;
    px = fmaf(K1, gx32, fmaf(c, dx, px));
    py = fmaf(K1, gy32, fmaf(c, dy, py));
    pz = fmaf(K1, gz32, fmaf(c, dz, pz));
}

// Plain Stokeslet pair in single precision (far zone of the mixed path).
__device__ __forceinline__ void far_pair32(float tx, float ty, float tz,
                                           float sx, float sy, float sz,
                                           float gx, float gy, float gz,
                                           float &ax, float &ay, float &az)
{
    const float dx = tx - sx, dy = ty - sy, dz = tz - sz;
    const float r2 = fmaf(dx, dx, fmaf(dy, dy, dz * dz));
    const float ri = __builtin_amdgcn_rsqf(r2);
    const float ri2 = ri * ri;
    const float gd = fmaf(gx, dx, fmaf(gy, dy, gz * dz));
    const float c = gd * ri2;
    ax = fmaf(ri, fmaf(c, dx, gx), ax);
    ay = fmaf(ri, fmaf(c, dy, gy), ay);
    az = fmaf(ri, fmaf(c, dz, gz), az);
}

// Knuth's two-sum: hi + lo accumulates s exactly up to the rounding of lo.
__device__ __forceinline__ void two_sum_acc(float s, float &hi, float &lo)
{
    const float t = hi + s;
    const float bp = t - hi;
    const float e = (hi - (t - bp)) + (s - bp);
    hi = t;
    lo += e;
}

// Per target block: bounding-sphere centre and radius and the far threshold cut * delta_max
// (the serving path keeps one threshold per precision in gap_far / gap_far_mixed).
struct TBlockRec {
    double cx, cy, cz, rad, gap_far, gap_far_mixed, pad0, pad1;
};

// Classification of a source cluster (bounding sphere S) against a target block: far when the
// gap between the spheres is at least `gap_far`.  Written with explicit fused operations only,
// so that every kernel that inlines it computes bit-identical gaps.
__device__ __forceinline__ bool cluster_is_far(const TBlockRec &tb, const double4 &S, double gap_far)
{
    const double ex = tb.cx - S.x, ey = tb.cy - S.y, ez = tb.cz - S.z;
    const double d2 = fma(ex, ex, fma(ey, ey, __dmul_rn(ez, ez)));
    const double gap = __dsub_rn(__dsub_rn(sqrt(d2), tb.rad), S.w);
    return gap >= gap_far;
}
__device__ __forceinline__ bool cluster_is_far(const TBlockRec &tb, const double4 &S)
{
    return cluster_is_far(tb, S, tb.gap_far);
}

// Wave-wide reductions (all 64 lanes active).
__device__ __forceinline__ double wave_min(double v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmin(v, __shfl_xor(v, o, kWave));
    return v;
}
__device__ __forceinline__ double wave_max(double v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, kWave));
    return v;
}
// Broadcast lane 0's value so the compiler treats it as wave-uniform (scalar register).
__device__ __forceinline__ double uniform(double v)
{
    const uint64_t b = __double_as_longlong(v);
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)b);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(b >> 32));
    return __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
}

}  // namespace sl
