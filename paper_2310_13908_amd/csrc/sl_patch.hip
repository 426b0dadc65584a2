// sl_patch.hip -- the per-patch regularization parameter of Sec. 3.4, eq. (regparam):
// delta = C delta*_i for every node of patch i, delta*_i the largest distance between two
// nodes of patch i that are adjacent in its grid (row, column or diagonal neighbours; a node on
// the edge of the grid has only the neighbours the grid holds).
//
// Each patch is split by rows over S workgroups (k_patch_max), whose maxima one workgroup per
// patch combines and writes out (k_patch_fill).  Every unordered adjacent pair is visited once,
// from its first node through the forward stencil (0, +1), (+1, -1), (+1, 0), (+1, +1); the
// squared distance is formed as ((dx dx + dy dy) + dz dz) with separately rounded operations,
// and the maximum of the squares is taken before the one square root, rounded to nearest
// (sqrt_rn; the rounded square root is monotone, so this equals the maximum of the rounded
// distances).  Maxima are order-independent, so the result is deterministic and equal to a
// plain double loop over the definition.
#include <algorithm>

#include "sl_internal.h"

namespace sl {

namespace {

constexpr int kPatchThreads = 1024;

// sqrt(t) rounded to nearest, for t >= 0: the hardware-based square root, then corrected with
// Tuckerman's test (y is the rounded root iff y y- < t <= y y+, y-/y+ its neighbours), whose
// products are signed exactly by fused multiply-adds.
__device__ double sqrt_rn(double t)
{
    double y = sqrt(t);
    if (!(y > 0.0)) return y;
    for (int k = 0; k < 2; ++k) {
        const double lo = __longlong_as_double(__double_as_longlong(y) - 1);
        const double hi = __longlong_as_double(__double_as_longlong(y) + 1);
        if (fma(y, lo, -t) >= 0.0) y = lo;
        else if (fma(y, hi, -t) < 0.0) y = hi;
        else break;
    }
    return y;
}

// Largest squared adjacent-pair distance over the rows of one part of a patch: blockIdx.x =
// patch i * S + part b; part b takes rows b, b + S, ...  The part's maximum goes to
// out[i n^2 + b] (the output doubles as scratch; n^2 >= S).
__global__ __launch_bounds__(kPatchThreads) void k_patch_max(int64_t n, int S, const double *__restrict__ x,
                                                             const double *__restrict__ y,
                                                             const double *__restrict__ z,
                                                             double *__restrict__ out)
{
#pragma clang fp contract(off)   // separately rounded products and sums, as the definition reads
    __shared__ double red[kPatchThreads / kWave];
    const int64_t i = blockIdx.x / S, b = blockIdx.x % S;
    const int64_t base = i * n * n;
    double m2 = 0.0;
    const int64_t rows = (n - b + S - 1) / S;
    for (int64_t f = threadIdx.x; f < rows * n; f += kPatchThreads) {
        const int64_t l = b + (f / n) * S, lp = f % n;
        const int64_t p = base + l * n + lp;
        const double px = x[p], py = y[p], pz = z[p];
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            const int64_t ql = s == 0 ? l : l + 1;
            const int64_t qlp = s == 0 ? lp + 1 : lp + (s - 2);
            if (ql >= n || qlp < 0 || qlp >= n) continue;
            const int64_t q = base + ql * n + qlp;
            const double dx = px - x[q], dy = py - y[q], dz = pz - z[q];
            const double d2 = (dx * dx + dy * dy) + dz * dz;
            m2 = fmax(m2, d2);
        }
    }
    m2 = wave_max(m2);
    if (threadIdx.x % kWave == 0) red[threadIdx.x / kWave] = m2;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int k = 0; k < kPatchThreads / kWave; ++k) t = fmax(t, red[k]);
        out[base + b] = t;
    }
}

// One workgroup per patch: the maximum of its S parts, then C sqrt(max) into every node.  The
// parts are read before the barrier that precedes any write.
__global__ __launch_bounds__(kPatchThreads) void k_patch_fill(int64_t n, int S, double C,
                                                              double *__restrict__ out)
{
    const int64_t base = (int64_t)blockIdx.x * n * n;
    double t = 0.0;
    for (int b = 0; b < S; ++b) t = fmax(t, out[base + b]);
    __syncthreads();
    const double d = C * sqrt_rn(t);
    for (int64_t p = threadIdx.x; p < n * n; p += kPatchThreads) out[base + p] = d;
}

}  // namespace

hipError_t launch_patch_delta(int64_t n_patches, int64_t n, const double *x, const double *y,
                              const double *z, double C, double *out, hipStream_t st)
{
    // parts per patch: enough workgroups to spread the patch over the chip, at most n rows
    int S = (int)std::min<int64_t>(n, std::max<int64_t>(1, n * n / 512));
    S = std::min(S, 64);
    hipLaunchKernelGGL(k_patch_max, dim3((unsigned)(n_patches * S)), dim3(kPatchThreads), 0, st, n, S, x, y,
                       z, out);
    hipLaunchKernelGGL(k_patch_fill, dim3((unsigned)n_patches), dim3(kPatchThreads), 0, st, n, S, C, out);
    return hipGetLastError();
}

}  // namespace sl
