// sl_pair.hip -- the O(N_t N_s) pair kernels of the regularized single layer (Sec. 3.4,
// eq. (regstokes)) on the gfx950 vector ALUs.
//
// Work decomposition.  One wavefront owns a block of 64 R consecutive (spatially sorted)
// targets, R per lane, held in registers, and sweeps one split of the source clusters.
// Source data are wave-uniform: every lane needs the same source at the same time, so the
// sources are read with scalar loads into scalar registers straight from L2 -- no LDS
// staging, no barriers, and every VALU instruction takes the source as a scalar operand.
// Per cluster of 64 sources the wave tests its bounding sphere against the target block's
// sphere (a uniform branch):
//   far  (gap >= cut * delta_max): plain Stokeslet, 28 flops a pair, no erf/exp.
//        FP64 path: double precision.  Mixed path: single precision, summed per cluster and
//        folded into a per-target two-sum (hi, lo) pair.
//   near: regularized kernel in double precision for every pair of the cluster; the
//        erf/exp smoothing runs only in lanes whose pair is within 6.9 delta.
// The FP64 far cut is 6.9 (s = 1 to double precision), the mixed one rho64 >= 5 (s = 1 to
// single precision).  Splits write unscaled partial sums; k_reduce adds them in a fixed
// order, scales by 1/(8 pi mu) and scatters to the caller's target order.
#include "sl_internal.h"

namespace sl {

namespace {

constexpr int kMinClustersPerSplit = 4;

template <int R, bool MIXED, bool VARD>
__global__ __launch_bounds__(kWave) void k_pair(PairArgs a)
{
    const int split = (int)(blockIdx.x % (unsigned)a.n_splits);
    const int tb = (int)(blockIdx.x / (unsigned)a.n_splits);
    const int lane = threadIdx.x;
    const int64_t t0 = (int64_t)tb * (kWave * R);
    const int64_t np_t = a.t.np;

    double tx[R], ty[R], tz[R];
    float tx32[R], ty32[R], tz32[R];
    DeltaC dcv[R];
    double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    double dmax = a.delta;
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int64_t i = t0 + r * kWave + lane;
        tx[r] = a.t.x[i];
        ty[r] = a.t.y[i];
        tz[r] = a.t.z[i];
        if constexpr (MIXED) {
            tx32[r] = a.t.x32[i];
            ty32[r] = a.t.y32[i];
            tz32[r] = a.t.z32[i];
        }
        if constexpr (VARD) {
            const double d = a.t.delta[i];
            dcv[r] = make_delta(d);
            dmax = r == 0 ? d : fmax(dmax, d);
        }
        lo[0] = fmin(lo[0], tx[r]); hi[0] = fmax(hi[0], tx[r]);
        lo[1] = fmin(lo[1], ty[r]); hi[1] = fmax(hi[1], ty[r]);
        lo[2] = fmin(lo[2], tz[r]); hi[2] = fmax(hi[2], tz[r]);
    }
    // Target-block bounding sphere and largest delta, made wave-uniform.
    const double cx = uniform(0.5 * (wave_min(lo[0]) + wave_max(hi[0])));
    const double cy = uniform(0.5 * (wave_min(lo[1]) + wave_max(hi[1])));
    const double cz = uniform(0.5 * (wave_min(lo[2]) + wave_max(hi[2])));
    double rr = 0.0;
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const double dx = tx[r] - cx, dy = ty[r] - cy, dz = tz[r] - cz;
        rr = fmax(rr, dx * dx + dy * dy + dz * dz);
    }
    const double trad = uniform(sqrt(wave_max(rr)) * (1.0 + 0x1p-40));
    if constexpr (VARD) dmax = uniform(wave_max(dmax));
    double gap_far = a.far_cut * dmax;
    if constexpr (MIXED) {
        // Single-precision positions carry an absolute error of about 2^-24 times the box
        // size; keep pairs closer than 2^-10 box sizes in double precision so that the
        // single-precision distance stays accurate (and never rounds to zero).
        const double bx = a.bbox[3] - a.bbox[0], by = a.bbox[4] - a.bbox[1], bz = a.bbox[5] - a.bbox[2];
        gap_far = fmax(gap_far, 0x1p-10 * sqrt(bx * bx + by * by + bz * bz));
    }
    const DeltaC dcu = make_delta(a.delta);

    double ax[R], ay[R], az[R];
    float hx[R], hy[R], hz[R], lx[R], ly[R], lz[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        ax[r] = ay[r] = az[r] = 0.0;
        hx[r] = hy[r] = hz[r] = lx[r] = ly[r] = lz[r] = 0.0f;
    }

    const int64_t n_cl = a.s.np / kCluster;
    const int64_t c_begin = (int64_t)split * a.clusters_per_split;
    const int64_t c_end = c_begin + a.clusters_per_split < n_cl ? c_begin + a.clusters_per_split : n_cl;
    for (int64_t c = c_begin; c < c_end; ++c) {
        const double4 S = a.s.sphere[c];
        const double ex = cx - S.x, ey = cy - S.y, ez = cz - S.z;
        const double gap = sqrt(ex * ex + ey * ey + ez * ez) - trad - S.w;
        const int64_t j0 = c * kCluster;
        if (gap >= gap_far) {
            if constexpr (MIXED) {
                float px[R], py[R], pz[R];
#pragma unroll
                for (int r = 0; r < R; ++r) px[r] = py[r] = pz[r] = 0.0f;
#pragma unroll 8
                for (int j = 0; j < kCluster; ++j) {
                    const float sx = a.s.x32[j0 + j], sy = a.s.y32[j0 + j], sz = a.s.z32[j0 + j];
                    const float gx = a.s.gx32[j0 + j], gy = a.s.gy32[j0 + j], gz = a.s.gz32[j0 + j];
#pragma unroll
                    for (int r = 0; r < R; ++r)
                        far_pair32(tx32[r], ty32[r], tz32[r], sx, sy, sz, gx, gy, gz, px[r], py[r], pz[r]);
                }
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    two_sum_acc(px[r], hx[r], lx[r]);
                    two_sum_acc(py[r], hy[r], ly[r]);
                    two_sum_acc(pz[r], hz[r], lz[r]);
                }
            } else {
#pragma unroll 4
                for (int j = 0; j < kCluster; ++j) {
                    const double sx = a.s.x[j0 + j], sy = a.s.y[j0 + j], sz = a.s.z[j0 + j];
                    const double gx = a.s.gx[j0 + j], gy = a.s.gy[j0 + j], gz = a.s.gz[j0 + j];
#pragma unroll
                    for (int r = 0; r < R; ++r)
                        far_pair64(tx[r], ty[r], tz[r], sx, sy, sz, gx, gy, gz, ax[r], ay[r], az[r]);
                }
            }
        } else {
#pragma unroll 1
            for (int j = 0; j < kCluster; ++j) {
                const double sx = a.s.x[j0 + j], sy = a.s.y[j0 + j], sz = a.s.z[j0 + j];
                const double gx = a.s.gx[j0 + j], gy = a.s.gy[j0 + j], gz = a.s.gz[j0 + j];
#pragma unroll
                for (int r = 0; r < R; ++r)
                    near_pair64(tx[r], ty[r], tz[r], sx, sy, sz, gx, gy, gz, VARD ? dcv[r] : dcu,
                                ax[r], ay[r], az[r]);
            }
        }
    }

    double *px = a.part + ((int64_t)split * 3 + 0) * np_t;
    double *py = a.part + ((int64_t)split * 3 + 1) * np_t;
    double *pz = a.part + ((int64_t)split * 3 + 2) * np_t;
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int64_t i = t0 + r * kWave + lane;
        double vx = ax[r], vy = ay[r], vz = az[r];
        if constexpr (MIXED) {
            vx += (double)hx[r] + (double)lx[r];
            vy += (double)hy[r] + (double)ly[r];
            vz += (double)hz[r] + (double)lz[r];
        }
        px[i] = vx;
        py[i] = vy;
        pz[i] = vz;
    }
}

__global__ __launch_bounds__(256) void k_reduce(const double *__restrict__ part, int n_splits,
                                                int64_t np, const int32_t *__restrict__ perm,
                                                double scale, double *__restrict__ ux,
                                                double *__restrict__ uy, double *__restrict__ uz)
{
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= np) return;
    const int32_t idx = perm[p];
    if (idx < 0) return;
    double a = 0.0, b = 0.0, c = 0.0;
    for (int s = 0; s < n_splits; ++s) {
        a += part[((int64_t)s * 3 + 0) * np + p];
        b += part[((int64_t)s * 3 + 1) * np + p];
        c += part[((int64_t)s * 3 + 2) * np + p];
    }
    ux[idx] = a * scale;
    uy[idx] = b * scale;
    uz[idx] = c * scale;
}

__global__ __launch_bounds__(256) void k_fill_zero(double *__restrict__ ux, double *__restrict__ uy,
                                                   double *__restrict__ uz, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) { ux[i] = 0.0; uy[i] = 0.0; uz[i] = 0.0; }
}

template <int R, bool MIXED, bool VARD>
hipError_t launch_t(const PairArgs &a, unsigned grid, hipStream_t st)
{
    hipLaunchKernelGGL((k_pair<R, MIXED, VARD>), dim3(grid), dim3(kWave), 0, st, a);
    return hipGetLastError();
}

template <int R>
hipError_t launch_r(const PairArgs &a, unsigned grid, bool mixed, bool vard, hipStream_t st)
{
    if (mixed) return vard ? launch_t<R, true, true>(a, grid, st) : launch_t<R, true, false>(a, grid, st);
    return vard ? launch_t<R, false, true>(a, grid, st) : launch_t<R, false, false>(a, grid, st);
}

}  // namespace

PairPlan plan_pairs(int64_t np_src, int64_t np_tgt, int R, int waves_wanted)
{
    PairPlan p;
    p.R = R;
    p.n_tblocks = (int)(np_tgt / (kWave * R));
    const int64_t n_cl = np_src / kCluster;
    int64_t S = (waves_wanted + p.n_tblocks - 1) / p.n_tblocks;
    const int64_t smax = n_cl / kMinClustersPerSplit > 0 ? n_cl / kMinClustersPerSplit : 1;
    S = S < 1 ? 1 : (S > smax ? smax : S);
    p.clusters_per_split = (n_cl + S - 1) / S;
    p.n_splits = (int)((n_cl + p.clusters_per_split - 1) / p.clusters_per_split);
    return p;
}

hipError_t launch_pair(const PairArgs &a, const PairPlan &p, bool mixed, bool var_delta,
                       hipStream_t st)
{
    const unsigned grid = (unsigned)((int64_t)p.n_tblocks * p.n_splits);
    switch (p.R) {
    case 1: return launch_r<1>(a, grid, mixed, var_delta, st);
    case 2: return launch_r<2>(a, grid, mixed, var_delta, st);
    case 4: return launch_r<4>(a, grid, mixed, var_delta, st);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_reduce(const double *part, int n_splits, int64_t np, const int32_t *perm,
                         double scale, double *ux, double *uy, double *uz, hipStream_t st)
{
    hipLaunchKernelGGL(k_reduce, dim3((unsigned)((np + 255) / 256)), dim3(256), 0, st, part,
                       n_splits, np, perm, scale, ux, uy, uz);
    return hipGetLastError();
}

hipError_t launch_fill_zero(double *ux, double *uy, double *uz, int64_t n, hipStream_t st)
{
    hipLaunchKernelGGL(k_fill_zero, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, ux, uy,
                       uz, n);
    return hipGetLastError();
}

}  // namespace sl
