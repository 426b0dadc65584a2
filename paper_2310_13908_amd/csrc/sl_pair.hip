// sl_pair.hip -- the O(N_t N_s) pair kernels of the regularized single layer (Sec. 3.4,
// eq. (regstokes)) on the gfx950 vector ALUs.
//
// Work decomposition.  One wavefront owns a block of 64 R consecutive (spatially sorted)
// targets, R per lane, held in registers, and sweeps one split of the source clusters.
// Source data are wave-uniform: every lane needs the same source at the same time, so the
// sources are read with scalar loads into scalar registers straight from L2 -- no LDS
// staging, no barriers, and every VALU instruction takes the source as a scalar operand.
//
// Each (target block, source cluster) pair is classified once by the bounding spheres:
//   far  (gap >= cut * delta_max): plain Stokeslet, 28 flops a pair, no erf/exp;
//   near: regularized kernel in double precision.
// Far and near clusters run in two kernels so that the far kernel -- the bulk of the work at
// large N -- carries none of the registers of the smoothing code and keeps a high occupancy:
//   k_tblock: per target block, bounding sphere and far threshold (read by both kernels, so
//             both classify every cluster from the same numbers);
//   k_far:    far clusters; FP64 path in double precision, mixed path in single precision
//             summed per cluster and folded into a per-target two-sum (hi, lo) pair;
//   k_near:   near clusters in double precision, added onto k_far's partial sums (same
//             stream, so the order of the additions is fixed);
//   k_reduce: adds the per-split partials in split order, scales by 1/(8 pi mu) and scatters
//             to the caller's target order.
// The FP64 far cut is 6.9 delta (s = 1 to double precision), the mixed one rho64 >= 5 (s = 1 to
// single precision), widened to 2^-10 box sizes so that single-precision distances stay exact
// enough.
#include "sl_internal.h"

namespace sl {

namespace {

constexpr int kMinClustersPerSplit = 4;
constexpr int kMaxNearWays = 64;

template <int R>
__global__ __launch_bounds__(kWave) void k_tblock(PairArgs a, TBlockRec *__restrict__ out,
                                                  int mixed, uint32_t *__restrict__ ctr)
{
    const int tb = blockIdx.x;
    const int lane = threadIdx.x;
    const int64_t t0 = (int64_t)tb * (kWave * R);
    double x[R], y[R], z[R];
    double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    double dmax = a.delta;
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int64_t i = t0 + r * kWave + lane;
        x[r] = a.t.x[i];
        y[r] = a.t.y[i];
        z[r] = a.t.z[i];
        if (a.t.delta) dmax = r == 0 ? a.t.delta[i] : fmax(dmax, a.t.delta[i]);
        lo[0] = fmin(lo[0], x[r]); hi[0] = fmax(hi[0], x[r]);
        lo[1] = fmin(lo[1], y[r]); hi[1] = fmax(hi[1], y[r]);
        lo[2] = fmin(lo[2], z[r]); hi[2] = fmax(hi[2], z[r]);
    }
    const double cx = 0.5 * (wave_min(lo[0]) + wave_max(hi[0]));
    const double cy = 0.5 * (wave_min(lo[1]) + wave_max(hi[1]));
    const double cz = 0.5 * (wave_min(lo[2]) + wave_max(hi[2]));
    double rr = 0.0;
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const double dx = x[r] - cx, dy = y[r] - cy, dz = z[r] - cz;
        rr = fmax(rr, fma(dx, dx, fma(dy, dy, __dmul_rn(dz, dz))));
    }
    rr = wave_max(rr);
    dmax = wave_max(dmax);
    if (lane == 0) {
        double gap_far = a.far_cut * dmax;
        if (mixed) {
            const double bx = a.bbox[3] - a.bbox[0], by = a.bbox[4] - a.bbox[1],
                         bz = a.bbox[5] - a.bbox[2];
            gap_far = fmax(gap_far, 0x1p-10 * sqrt(fma(bx, bx, fma(by, by, __dmul_rn(bz, bz)))));
        }
        TBlockRec rec;
        rec.cx = cx; rec.cy = cy; rec.cz = cz;
        rec.rad = sqrt(rr) * (1.0 + 0x1p-40);
        rec.gap_far = gap_far;
        rec.gap_far_mixed = gap_far;
        rec.pad0 = rec.pad1 = 0.0;
        out[tb] = rec;
        if (tb == 0) {          // work counters of k_far and k_near, which run after this kernel
            ctr[0] = 0u;
            ctr[1] = 0u;
        }
    }
}

// Far clusters of source split `split` against target block `tb`.  The source arrays arrive as
// separate restrict-qualified kernel arguments: the compiler then knows that the partial-sum
// stores never alias them and keeps reading them with scalar loads inside the work loop.
template <int R, bool MIXED>
__device__ __forceinline__ void far_item(const PairArgs &a, const TBlockRec *__restrict__ tbr,
                                         const double *__restrict__ Sx, const double *__restrict__ Sy,
                                         const double *__restrict__ Sz, const double *__restrict__ Gx,
                                         const double *__restrict__ Gy, const double *__restrict__ Gz,
                                         const float *__restrict__ Sx32, const float *__restrict__ Sy32,
                                         const float *__restrict__ Sz32, const float *__restrict__ Gx32,
                                         const float *__restrict__ Gy32, const float *__restrict__ Gz32,
                                         const double4 *__restrict__ sphere, double *__restrict__ part,
                                         int tb, int split)
{
    const int lane = threadIdx.x;
    const int64_t t0 = (int64_t)tb * (kWave * R);
    const int64_t np_t = a.t.np;
    const TBlockRec rec = tbr[tb];

    double tx[R], ty[R], tz[R];
    float tx32[R], ty32[R], tz32[R];
    double ax[R], ay[R], az[R];
    float hx[R], hy[R], hz[R], lx[R], ly[R], lz[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int64_t i = t0 + r * kWave + lane;
        if constexpr (MIXED) {
            tx32[r] = a.t.x32[i];
            ty32[r] = a.t.y32[i];
            tz32[r] = a.t.z32[i];
            hx[r] = hy[r] = hz[r] = lx[r] = ly[r] = lz[r] = 0.0f;
        } else {
            tx[r] = a.t.x[i];
            ty[r] = a.t.y[i];
            tz[r] = a.t.z[i];
            ax[r] = ay[r] = az[r] = 0.0;
        }
    }

    const int64_t n_cl = a.s.np / kCluster;
    const int64_t c_begin = (int64_t)split * a.clusters_per_split;
    const int64_t c_end = c_begin + a.clusters_per_split < n_cl ? c_begin + a.clusters_per_split : n_cl;
    for (int64_t c = c_begin; c < c_end; ++c) {
        if (!cluster_is_far(rec, sphere[c])) continue;
        const int64_t j0 = c * kCluster;
        if constexpr (MIXED) {
            float px[R], py[R], pz[R];
#pragma unroll
            for (int r = 0; r < R; ++r) px[r] = py[r] = pz[r] = 0.0f;
#pragma unroll 8
            for (int j = 0; j < kCluster; ++j) {
                const float sx = Sx32[j0 + j], sy = Sy32[j0 + j], sz = Sz32[j0 + j];
                const float gx = Gx32[j0 + j], gy = Gy32[j0 + j], gz = Gz32[j0 + j];
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
                const double sx = Sx[j0 + j], sy = Sy[j0 + j], sz = Sz[j0 + j];
                const double gx = Gx[j0 + j], gy = Gy[j0 + j], gz = Gz[j0 + j];
#pragma unroll
                for (int r = 0; r < R; ++r)
                    far_pair64(tx[r], ty[r], tz[r], sx, sy, sz, gx, gy, gz, ax[r], ay[r], az[r]);
            }
        }
    }

    double *px = part + ((int64_t)split * 3 + 0) * np_t;
    double *py = part + ((int64_t)split * 3 + 1) * np_t;
    double *pz = part + ((int64_t)split * 3 + 2) * np_t;
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int64_t i = t0 + r * kWave + lane;
        if constexpr (MIXED) {
            px[i] = (double)hx[r] + (double)lx[r];
            py[i] = (double)hy[r] + (double)ly[r];
            pz[i] = (double)hz[r] + (double)lz[r];
        } else {
            px[i] = ax[r];
            py[i] = ay[r];
            pz[i] = az[r];
        }
    }
}

// Next work item of a wave (lane 0 draws from the counter; the index is made wave-uniform).
__device__ __forceinline__ uint32_t next_item(uint32_t *__restrict__ ctr)
{
    uint32_t v = 0;
    if (threadIdx.x == 0) v = atomicAdd(ctr, 1u);
    return __builtin_amdgcn_readfirstlane(v);
}

// Occupancy-sized grid; every wave pulls (split, target block) items until none are left.
// Items are split-major, so the waves working at the same time share one source split in L2.
template <int R, bool MIXED>
__global__ __launch_bounds__(kWave) void k_far(PairArgs a, const TBlockRec *__restrict__ tbr,
                                               const double *__restrict__ Sx, const double *__restrict__ Sy,
                                               const double *__restrict__ Sz, const double *__restrict__ Gx,
                                               const double *__restrict__ Gy, const double *__restrict__ Gz,
                                               const float *__restrict__ Sx32, const float *__restrict__ Sy32,
                                               const float *__restrict__ Sz32, const float *__restrict__ Gx32,
                                               const float *__restrict__ Gy32, const float *__restrict__ Gz32,
                                               const double4 *__restrict__ sphere, double *__restrict__ part,
                                               uint32_t *__restrict__ ctr)
{
    const uint32_t n_items = (uint32_t)a.n_tblocks * (uint32_t)a.n_splits;
    for (uint32_t item = next_item(ctr); item < n_items; item = next_item(ctr)) {
        const int tb = (int)(item % (uint32_t)a.n_tblocks);
        const int split = (int)(item / (uint32_t)a.n_tblocks);
        far_item<R, MIXED>(a, tbr, Sx, Sy, Sz, Gx, Gy, Gz, Sx32, Sy32, Sz32, Gx32, Gy32, Gz32,
                           sphere, part, tb, split);
    }
}

// Near clusters of a target block are few and contiguous in the sorted order, so they are dealt
// out by rank instead of by source range: wave (tb, k) scans all clusters 64 at a time (one per
// lane), and takes the near clusters whose rank among the block's near clusters is k mod K.
// FP64 path: every pair in double precision.  Mixed path: near_pair_mixed (double precision only
// below rho64 delta); single-precision terms are summed per cluster and folded into a two-sum
// (hi, lo) pair per target, as in the far kernel.
template <int R, bool VARD, bool MIXED>
__device__ __forceinline__ void near_item(const PairArgs &a, const TBlockRec *__restrict__ tbr,
                                          const double *__restrict__ Sx, const double *__restrict__ Sy,
                                          const double *__restrict__ Sz, const double *__restrict__ Gx,
                                          const double *__restrict__ Gy, const double *__restrict__ Gz,
                                          const float *__restrict__ Sx32, const float *__restrict__ Sy32,
                                          const float *__restrict__ Sz32, const float *__restrict__ Gx32,
                                          const float *__restrict__ Gy32, const float *__restrict__ Gz32,
                                          const double4 *__restrict__ sphere,
                                          double *__restrict__ part_near, int tb, int k)
{
    const int K = a.near_ways;
    const int lane = threadIdx.x;
    const int64_t t0 = (int64_t)tb * (kWave * R);
    const int64_t np_t = a.t.np;
    const TBlockRec rec = tbr[tb];

    double tx[R], ty[R], tz[R], ax[R], ay[R], az[R];
    float tx32[R], ty32[R], tz32[R], hx[R], hy[R], hz[R], lx[R], ly[R], lz[R];
    DeltaC dcv[R];
    DeltaC32 dcv32[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int64_t i = t0 + r * kWave + lane;
        tx[r] = a.t.x[i];
        ty[r] = a.t.y[i];
        tz[r] = a.t.z[i];
        if constexpr (VARD) {
            dcv[r] = make_delta(a.t.delta[i]);
            if constexpr (MIXED) dcv32[r] = make_delta32(a.t.delta[i], a.rho64);
        }
        if constexpr (MIXED) {
            tx32[r] = a.t.x32[i];
            ty32[r] = a.t.y32[i];
            tz32[r] = a.t.z32[i];
        }
        ax[r] = ay[r] = az[r] = 0.0;
        hx[r] = hy[r] = hz[r] = lx[r] = ly[r] = lz[r] = 0.0f;
    }
    const DeltaC dcu = make_delta(a.delta);
    const DeltaC32 dcu32 = make_delta32(a.delta, a.rho64);

    const int64_t n_cl = a.s.np / kCluster;
    uint32_t rank = 0;
    for (int64_t c0 = 0; c0 < n_cl; c0 += kWave) {
        const int64_t cl = c0 + lane;
        const bool near = cl < n_cl && !cluster_is_far(rec, sphere[cl]);
        uint64_t mask = __ballot(near);
        while (mask) {
            const int b = __builtin_ctzll(mask);
            mask &= mask - 1;
            if ((int)(rank++ % (uint32_t)K) != k) continue;
            const int64_t j0 = (c0 + b) * kCluster;
            if constexpr (MIXED) {
                float px[R], py[R], pz[R];
#pragma unroll
                for (int r = 0; r < R; ++r) px[r] = py[r] = pz[r] = 0.0f;
#pragma unroll 4
                for (int j = 0; j < kCluster; ++j) {
                    const float sx32 = Sx32[j0 + j], sy32 = Sy32[j0 + j], sz32 = Sz32[j0 + j];
                    const float gx32 = Gx32[j0 + j], gy32 = Gy32[j0 + j], gz32 = Gz32[j0 + j];
                    const double sx = Sx[j0 + j], sy = Sy[j0 + j], sz = Sz[j0 + j];
                    const double gx = Gx[j0 + j], gy = Gy[j0 + j], gz = Gz[j0 + j];
#pragma unroll
                    for (int r = 0; r < R; ++r)
                        near_pair_mixed(tx32[r], ty32[r], tz32[r], tx[r], ty[r], tz[r], sx32, sy32,
                                        sz32, gx32, gy32, gz32, sx, sy, sz, gx, gy, gz,
                                        VARD ? dcv[r] : dcu, VARD ? dcv32[r] : dcu32, px[r], py[r],
                                        pz[r], ax[r], ay[r], az[r]);
                }
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    two_sum_acc(px[r], hx[r], lx[r]);
                    two_sum_acc(py[r], hy[r], ly[r]);
                    two_sum_acc(pz[r], hz[r], lz[r]);
                }
            } else {
#pragma unroll 2
                for (int j = 0; j < kCluster; ++j) {
                    const double sx = Sx[j0 + j], sy = Sy[j0 + j], sz = Sz[j0 + j];
                    const double gx = Gx[j0 + j], gy = Gy[j0 + j], gz = Gz[j0 + j];
#pragma unroll
                    for (int r = 0; r < R; ++r)
                        near_pair64(tx[r], ty[r], tz[r], sx, sy, sz, gx, gy, gz, VARD ? dcv[r] : dcu,
                                    ax[r], ay[r], az[r]);
                }
            }
        }
    }

    double *px = part_near + ((int64_t)k * 3 + 0) * np_t;
    double *py = part_near + ((int64_t)k * 3 + 1) * np_t;
    double *pz = part_near + ((int64_t)k * 3 + 2) * np_t;
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int64_t i = t0 + r * kWave + lane;
        px[i] = ax[r] + ((double)hx[r] + (double)lx[r]);
        py[i] = ay[r] + ((double)hy[r] + (double)ly[r]);
        pz[i] = az[r] + ((double)hz[r] + (double)lz[r]);
    }
}

// Occupancy-sized grid pulling (target block, way) items, block-major so that the waves of one
// block (which read the same near sources) run together.
template <int R, bool VARD, bool MIXED>
__global__ __launch_bounds__(kWave) void k_near(PairArgs a, const TBlockRec *__restrict__ tbr,
                                                const double *__restrict__ Sx, const double *__restrict__ Sy,
                                                const double *__restrict__ Sz, const double *__restrict__ Gx,
                                                const double *__restrict__ Gy, const double *__restrict__ Gz,
                                                const float *__restrict__ Sx32, const float *__restrict__ Sy32,
                                                const float *__restrict__ Sz32, const float *__restrict__ Gx32,
                                                const float *__restrict__ Gy32, const float *__restrict__ Gz32,
                                                const double4 *__restrict__ sphere,
                                                double *__restrict__ part_near, uint32_t *__restrict__ ctr)
{
    const uint32_t n_items = (uint32_t)a.n_tblocks * (uint32_t)a.near_ways;
    for (uint32_t item = next_item(ctr); item < n_items; item = next_item(ctr))
        near_item<R, VARD, MIXED>(a, tbr, Sx, Sy, Sz, Gx, Gy, Gz, Sx32, Sy32, Sz32, Gx32, Gy32, Gz32,
                                  sphere, part_near, (int)(item / (uint32_t)a.near_ways),
                                  (int)(item % (uint32_t)a.near_ways));
}

// Per target: far partials of the source splits, then near partials of the K ways, in order.
__global__ __launch_bounds__(256) void k_reduce(const double *__restrict__ part, int n_splits,
                                                const double *__restrict__ part_near, int near_ways,
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
    for (int s = 0; s < near_ways; ++s) {
        a += part_near[((int64_t)s * 3 + 0) * np + p];
        b += part_near[((int64_t)s * 3 + 1) * np + p];
        c += part_near[((int64_t)s * 3 + 2) * np + p];
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

// Resident wavefronts per CU of a kernel (queried once per kernel instance).
template <typename K>
int resident_waves(K kernel)
{
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, (const void *)kernel, kWave, 0) != hipSuccess ||
        nb < 1)
        nb = 4;
    return nb;
}

template <typename K>
unsigned work_grid(K kernel, int &cache, int n_cu, int64_t n_items)
{
    if (cache == 0) cache = resident_waves(kernel);
    const int64_t g = (int64_t)n_cu * cache;
    return (unsigned)(g < n_items ? g : n_items);
}

template <int R>
hipError_t launch_r(const PairArgs &a, const PairPlan &p, bool mixed, bool vard, hipStream_t st,
                    const PairTiming *tm)
{
    static int occ_far[2] = {0, 0}, occ_near[4] = {0, 0, 0, 0};
    TBlockRec *rec = reinterpret_cast<TBlockRec *>(a.tblock_scratch);
    uint32_t *ctr = reinterpret_cast<uint32_t *>(reinterpret_cast<char *>(a.tblock_scratch) +
                                                 tblock_scratch_bytes(p.n_tblocks) - 256);
    const SrcView &s = a.s;
    hipLaunchKernelGGL((k_tblock<R>), dim3(p.n_tblocks), dim3(kWave), 0, st, a, rec, (int)mixed, ctr);
    if (tm && tm->e0) (void)hipEventRecord(tm->e0, st);
    const int64_t n_far = (int64_t)p.n_tblocks * p.n_splits;
    if (mixed)
        hipLaunchKernelGGL((k_far<R, true>), dim3(work_grid(k_far<R, true>, occ_far[1], p.n_cu, n_far)),
                           dim3(kWave), 0, st, a, rec, s.x, s.y, s.z, s.gx, s.gy, s.gz, s.x32, s.y32,
                           s.z32, s.gx32, s.gy32, s.gz32, s.sphere, a.part, ctr);
    else
        hipLaunchKernelGGL((k_far<R, false>), dim3(work_grid(k_far<R, false>, occ_far[0], p.n_cu, n_far)),
                           dim3(kWave), 0, st, a, rec, s.x, s.y, s.z, s.gx, s.gy, s.gz, s.x32, s.y32,
                           s.z32, s.gx32, s.gy32, s.gz32, s.sphere, a.part, ctr);
    if (tm && tm->e1) (void)hipEventRecord(tm->e1, st);
    const int64_t n_near = (int64_t)p.n_tblocks * p.near_ways;
#define SL_NEAR_LAUNCH(V, M, SLOT)                                                                  \
    hipLaunchKernelGGL((k_near<R, V, M>), dim3(work_grid(k_near<R, V, M>, occ_near[SLOT], p.n_cu, n_near)), \
                       dim3(kWave), 0, st, a, rec, s.x, s.y, s.z, s.gx, s.gy, s.gz, s.x32, s.y32, s.z32, \
                       s.gx32, s.gy32, s.gz32, s.sphere, a.part_near, ctr + 1)
    if (vard) {
        if (mixed) SL_NEAR_LAUNCH(true, true, 3); else SL_NEAR_LAUNCH(true, false, 1);
    } else {
        if (mixed) SL_NEAR_LAUNCH(false, true, 2); else SL_NEAR_LAUNCH(false, false, 0);
    }
#undef SL_NEAR_LAUNCH
    if (tm && tm->e2) (void)hipEventRecord(tm->e2, st);
    return hipGetLastError();
}

}  // namespace

// Target-block records followed by 256 bytes holding the two work counters.
size_t tblock_scratch_bytes(int n_tblocks) { return (size_t)n_tblocks * sizeof(TBlockRec) + 256; }

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
    int64_t K = (waves_wanted + p.n_tblocks - 1) / p.n_tblocks;
    K = K < 1 ? 1 : (K > kMaxNearWays ? kMaxNearWays : K);
    K = K > n_cl ? n_cl : K;
    p.near_ways = (int)K;
    return p;
}

hipError_t launch_pair(const PairArgs &a, const PairPlan &p, bool mixed, bool var_delta,
                       hipStream_t st, const PairTiming *tm)
{
    switch (p.R) {
    case 1: return launch_r<1>(a, p, mixed, var_delta, st, tm);
    case 2: return launch_r<2>(a, p, mixed, var_delta, st, tm);
    case 4: return launch_r<4>(a, p, mixed, var_delta, st, tm);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_reduce(const double *part, int n_splits, const double *part_near, int near_ways,
                         int64_t np, const int32_t *perm, double scale, double *ux, double *uy,
                         double *uz, hipStream_t st)
{
    hipLaunchKernelGGL(k_reduce, dim3((unsigned)((np + 255) / 256)), dim3(256), 0, st, part,
                       n_splits, part_near, near_ways, np, perm, scale, ux, uy, uz);
    return hipGetLastError();
}

hipError_t launch_fill_zero(double *ux, double *uy, double *uz, int64_t n, hipStream_t st)
{
    hipLaunchKernelGGL(k_fill_zero, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, ux, uy,
                       uz, n);
    return hipGetLastError();
}

}  // namespace sl
