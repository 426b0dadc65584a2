// sl_device.h -- device arithmetic of the regularized Stokes single layer on gfx950.
//
// Pair term (Sec. 3.4, eq. (regstokes)), for target t, source x with packed density
// g = w f (the trapezoid-POU weight of Sec. 3.3 folded into the force), d = t - x, r = |d|:
//
//     term = K1 g + K2 (g . d) d,   K1 = s1(r/delta)/r,  K2 = s2(r/delta)/r^3.
//
// Far from the target (r/delta >= 6.9) both smoothing factors equal 1 to double precision
// (|s - 1| < 2^-53; at r/delta >= 5, |s - 1| < 2^-24), so the far pair is the plain
// Stokeslet K1 = 1/r, K2 = 1/r^3: 28 flops, no erf/exp.  Near the target the smoothing is
// applied in double precision, written without divisions:
//
//     q = (r/delta)^2,  E = exp(-q),  a = (2/(3 sqrt(pi))) E / delta,
//     K1 = erf(r/delta)/r - a (2q - 5),
//     K2 = erf(r/delta)/r^3 - a ( (4q - 14)/delta^2 + 3/r^2 ),
//
// which is s1/r and s2/r^3 of Sec. 3.4 expanded; at r = 0 the limit K1 = 16/(3 delta sqrt(pi))
// of Sec. 3.4 is used (the K2 term carries d twice and vanishes).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace sl {

constexpr int kWave = 64;            // CDNA wavefront width
constexpr int kCluster = 64;         // sources per cluster (one classification unit)
constexpr int kPad = 256;            // point arrays are padded to a multiple of this
constexpr double kC0 = 0.376126389031837524632052967707181724;   // 2 / (3 sqrt(pi))
constexpr double kRhoExact64 = 6.9;  // s1 = s2 = 1 in double precision beyond this r/delta
constexpr double kRhoExact32 = 5.0;  // ... and in single precision beyond this r/delta

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

// Per-target constants of the smoothing: 1/delta, 1/delta^2, a0 = 2/(3 sqrt(pi) delta) and
// the squared radius inside which the smoothing differs from 1 in double precision.
struct DeltaC {
    double id, id2, a0, cut2;
};

__device__ __forceinline__ DeltaC make_delta(double delta)
{
    DeltaC c;
    c.id = 1.0 / delta;
    c.id2 = c.id * c.id;
    c.a0 = kC0 * c.id;
    const double rc = kRhoExact64 * delta;
    c.cut2 = rc * rc;
    return c;
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
    const bool pos = r2 > 0.0;
    const double ri = rsqrt64(pos ? r2 : 1.0);
    const double ri2 = ri * ri;
    double K1 = ri, K2 = ri * ri2;
    if (r2 < dc.cut2) {
        const double q = r2 * dc.id2;
        const double rho = (r2 * ri) * dc.id;
        const double a = dc.a0 * exp(-q);
        const double er = erf(rho);
        K1 = fma(-a, fma(2.0, q, -5.0), er * ri);
        K2 = fma(-a, fma(dc.id2, fma(4.0, q, -14.0), 3.0 * ri2), er * ri * ri2);
        if (!pos) {
            K1 = 8.0 * dc.a0;       // 16 / (3 sqrt(pi) delta)
            K2 = 0.0;
        }
    }
    const double gd = fma(gx, dx, fma(gy, dy, gz * dz));
    const double c = gd * K2;
    ax = fma(K1, gx, fma(c, dx, ax));
    ay = fma(K1, gy, fma(c, dy, ay));
    az = fma(K1, gz, fma(c, dz, az));
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
