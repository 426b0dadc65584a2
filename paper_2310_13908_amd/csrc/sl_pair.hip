// sl_pair.hip -- the O(N_t N_s) pair kernel of the regularized single layer (Sec. 3.4,
// eq. (regstokes)) on the gfx950 vector ALUs.
//
// Work decomposition.  One wavefront owns a block of 64 R consecutive (spatially sorted)
// targets, R per lane, held in registers.  Source data are wave-uniform: every lane needs the
// same source at the same time.  The mixed kernel without the double-precision zone copies each
// cluster it walks into the wave's own LDS area and reads every record back as a broadcast, so
// that its single-precision instructions take the source as a vector operand (a scalar operand
// halves their issue rate); the other kernels read sources with scalar loads into scalar
// registers.  The G waves of a workgroup (mixed path) own G adjacent target blocks and walk the
// same source clusters, so a record fetched by one of them is in cache for the others.
//
// Each (target group, source cluster of 64) pair is classified once by the bounding spheres:
//   far  (gap >= cut * delta_max): plain Stokeslet, 28 flops a pair, no erf/exp;
//   near: regularized kernel (double precision, or the mixed path's single-precision table with
//         an optional double-precision zone), with the smoothing evaluated only where some lane
//         of the wavefront needs it.
// The clusters of a group are dealt out to K ways by rank among the group's far clusters and,
// separately, among its near clusters, so that every way of every group carries the same work
// to within one cluster of each kind, whatever the geometry; the K partial sums per target are
// added in a fixed order afterwards, so the result is deterministic.
//   mixed path: way k takes the ranks in [k n / K, (k + 1) n / K) of each kind (n: the group's
//     count of that kind), and the work items run way by way.  The items in flight at any time
//     then read about 1/K of the source records, which stay in each XCD's L2: at 6 x 256^2
//     points this cuts the kernel's fetches from memory twelvefold, at the same speed.
//   FP64 path: way k takes the ranks congruent to k mod K, and the items run group by group.
//     Contiguous ranges measured slower here (7% at 6 x 256^2 points with the items way by way,
//     10% group by group, 16% at 6 x 64^2): a way's near clusters then come in one spatial run,
//     so the closest ones, where most pairs need the smoothing, fall to few ways; the interleaved
//     deal keeps every way's mix even.
//   k_tblock: per target group, bounding sphere and far threshold;
//   k_counts: per target group, the numbers of far and near clusters (mixed path);
//   k_pair:   occupancy-sized grid; every workgroup pulls work items off a counter;
//   k_reduce: adds the K partials of each target in way order, scales by 1/(8 pi mu) and
//             scatters to the caller's target order.
// The FP64 far cut is 6.9 delta (s = 1 to double precision), the mixed one max(rho64, 5) (s = 1
// to single precision), widened to 2^-10 box sizes so that single-precision distances stay
// accurate enough.
#include "sl_internal.h"

namespace sl {

namespace {

// Most ways per target block.  The mixed kernel is fast enough that the K per-way partial sums
// (K x 3 x 8 bytes per target, written and read back once) weigh against finer items sooner.
constexpr int kMaxWays = 128;
constexpr int kMaxWaysMixed = 64;

__device__ __forceinline__ TBlockRec make_rec(const PairArgs &a, int mixed, double cx, double cy,
                                              double cz, double rad, double dmax)
{
    double gap_far = a.far_cut * dmax;
    if (mixed) {
        const double bx = a.bbox[3] - a.bbox[0], by = a.bbox[4] - a.bbox[1], bz = a.bbox[5] - a.bbox[2];
        gap_far = fmax(gap_far, 0x1p-10 * sqrt(fma(bx, bx, fma(by, by, __dmul_rn(bz, bz)))));
    }
    TBlockRec rec;
    rec.cx = cx; rec.cy = cy; rec.cz = cz;
    rec.rad = rad;
    rec.gap_far = gap_far;
    rec.gap_far_mixed = gap_far;
    rec.pad0 = rec.pad1 = 0.0;
    return rec;
}

// Sphere (centre of the box, farthest member, relative margin 2^-40) and far threshold of each
// group of G target blocks (G * 64 R consecutive sorted targets; the last group may be short)
// and, when G > 1, of each of its blocks.  One workgroup per group, wave w on block G g + w.
// Records: [n_groups] group records, then [n_tblocks] block records.
template <int R, int G>
__global__ __launch_bounds__(G * kWave) void k_tblock(PairArgs a, TBlockRec *__restrict__ out,
                                                      int mixed, uint32_t *__restrict__ ctr)
{
    __shared__ double sh[G][8];
    const int g = blockIdx.x;
    const int w = threadIdx.x / kWave, lane = threadIdx.x % kWave;
    const int n_groups = (a.n_tblocks + G - 1) / G;
    const int b = g * G + w;
    const int64_t blk = (int64_t)kWave * R;
    const int64_t t0 = b < a.n_tblocks ? (int64_t)b * blk : 0;
    const int64_t t1 = b < a.n_tblocks ? t0 + blk : 0;
    double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    double dmax = a.t.delta ? 0.0 : a.delta;
    for (int64_t i = t0 + lane; i < t1; i += kWave) {
        const double x = a.t.x[i], y = a.t.y[i], z = a.t.z[i];
        if (a.t.delta) dmax = fmax(dmax, a.t.delta[i]);
        lo[0] = fmin(lo[0], x); hi[0] = fmax(hi[0], x);
        lo[1] = fmin(lo[1], y); hi[1] = fmax(hi[1], y);
        lo[2] = fmin(lo[2], z); hi[2] = fmax(hi[2], z);
    }
#pragma unroll
    for (int k = 0; k < 3; ++k) { lo[k] = wave_min(lo[k]); hi[k] = wave_max(hi[k]); }
    dmax = wave_max(dmax);
    if (lane == 0) {
        for (int k = 0; k < 3; ++k) { sh[w][k] = lo[k]; sh[w][3 + k] = hi[k]; }
        sh[w][6] = dmax;
    }
    __syncthreads();
    double glo[3] = {INFINITY, INFINITY, INFINITY}, ghi[3] = {-INFINITY, -INFINITY, -INFINITY};
    double gdmax = 0.0;
    for (int v = 0; v < G; ++v)
        if (g * G + v < a.n_tblocks) {
            for (int k = 0; k < 3; ++k) { glo[k] = fmin(glo[k], sh[v][k]); ghi[k] = fmax(ghi[k], sh[v][3 + k]); }
            gdmax = fmax(gdmax, sh[v][6]);
        }
    const double gx = 0.5 * (glo[0] + ghi[0]), gy = 0.5 * (glo[1] + ghi[1]), gz = 0.5 * (glo[2] + ghi[2]);
    const double cx = 0.5 * (lo[0] + hi[0]), cy = 0.5 * (lo[1] + hi[1]), cz = 0.5 * (lo[2] + hi[2]);
    double rr = 0.0, grr = 0.0;
    for (int64_t i = t0 + lane; i < t1; i += kWave) {
        const double x = a.t.x[i], y = a.t.y[i], z = a.t.z[i];
        const double dx = x - cx, dy = y - cy, dz = z - cz;
        rr = fmax(rr, fma(dx, dx, fma(dy, dy, __dmul_rn(dz, dz))));
        const double ex = x - gx, ey = y - gy, ez = z - gz;
        grr = fmax(grr, fma(ex, ex, fma(ey, ey, __dmul_rn(ez, ez))));
    }
    rr = wave_max(rr);
    grr = wave_max(grr);
    __syncthreads();                 // everyone has read sh[][0..6]
    if (lane == 0) sh[w][7] = grr;
    __syncthreads();
    if (threadIdx.x == 0) {
        double gr = 0.0;
        for (int v = 0; v < G; ++v)
            if (g * G + v < a.n_tblocks) gr = fmax(gr, sh[v][7]);
        out[g] = make_rec(a, mixed, gx, gy, gz, sqrt(gr) * (1.0 + 0x1p-40), gdmax);
        if (g == 0) ctr[0] = 0u;   // work counter of k_pair, which runs after this kernel
    }
    if (G > 1 && lane == 0 && b < a.n_tblocks)
        out[n_groups + b] = make_rec(a, mixed, cx, cy, cz, sqrt(rr) * (1.0 + 0x1p-40), dmax);
}

// Source records of the pair kernel ([np][8]: x, y, z, gx, gy, gz, 0, 0).  They arrive as
// restrict-qualified kernel arguments: the compiler then knows that the partial-sum stores
// never alias them and reads each record with wide scalar loads inside the work loop.
struct Src {
    const double *__restrict__ d;
    const float *__restrict__ f;
};

// Per-target state of one work item.
template <int R, bool VARD, bool MIXED>
struct Acc {
    double tx[R], ty[R], tz[R];
    float tx32[R], ty32[R], tz32[R];
    double ax[R], ay[R], az[R];          // FP64 sums (mixed: the FP64 zone)
    float hx[R], hy[R], hz[R], lx[R], ly[R], lz[R];   // mixed: two-sum of per-cluster sums
    DeltaC dc[VARD ? R : 1];
    DeltaC32 dc32[VARD ? R : 1];
};

// Source record j of the cluster at j0 in single precision: from the wave's LDS copy of the
// cluster (STAGE) or, wave-uniform, from memory through scalar loads.
template <bool STAGE>
__device__ __forceinline__ void src32(const Src &S, int64_t j0, const float4 *stg, int j, float &sx,
                                      float &sy, float &sz, float &gx, float &gy, float &gz)
{
    if constexpr (STAGE) {
        const float4 u = stg[2 * j], v = stg[2 * j + 1];
        sx = u.x; sy = u.y; sz = u.z; gx = u.w; gy = v.x; gz = v.y;
    } else {
        const float *q = S.f + (j0 + j) * 8;
        sx = q[0]; sy = q[1]; sz = q[2]; gx = q[3]; gy = q[4]; gz = q[5];
    }
}

template <int R, bool VARD, bool MIXED, bool STAGE>
__device__ __forceinline__ void far_cluster(const Src &S, int64_t j0, const float4 *stg,
                                            Acc<R, VARD, MIXED> &A)
{
    if constexpr (MIXED) {
        float px[R], py[R], pz[R];
#pragma unroll
        for (int r = 0; r < R; ++r) px[r] = py[r] = pz[r] = 0.0f;
#pragma unroll 4
        for (int j = 0; j < kCluster; ++j) {
            float sx, sy, sz, gx, gy, gz;
            src32<STAGE>(S, j0, stg, j, sx, sy, sz, gx, gy, gz);
#pragma unroll
            for (int r = 0; r < R; ++r)
                far_pair32(A.tx32[r], A.ty32[r], A.tz32[r], sx, sy, sz, gx, gy, gz, px[r], py[r], pz[r]);
        }
#pragma unroll
        for (int r = 0; r < R; ++r) {
            two_sum_acc(px[r], A.hx[r], A.lx[r]);
            two_sum_acc(py[r], A.hy[r], A.ly[r]);
            two_sum_acc(pz[r], A.hz[r], A.lz[r]);
        }
    } else {
#pragma unroll 4
        for (int j = 0; j < kCluster; ++j) {
            const double *q = S.d + (j0 + j) * 8;
            const double sx = q[0], sy = q[1], sz = q[2], gx = q[3], gy = q[4], gz = q[5];
#pragma unroll
            for (int r = 0; r < R; ++r)
                far_pair64(A.tx[r], A.ty[r], A.tz[r], sx, sy, sz, gx, gy, gz, A.ax[r], A.ay[r], A.az[r]);
        }
    }
}

// FP64 path: every pair in double precision.  Mixed path: near_pair32 (the single-precision
// zones), summed per cluster and folded into the two-sum pair as for far clusters, and with
// ZONE the double-precision zone (pairs below rho64, zone_pair64), whose state lives in LDS
// (`zs`: per target of the lane, x, y, z and the three sums, 64 apart): it is needed only for
// the few sources with such a pair, and keeping it out of the vector registers buys the kernel
// a wave per SIMD.
template <int R, bool VARD, bool MIXED, bool ZONE, bool STAGE>
__device__ __forceinline__ void near_cluster(const Src &S, int64_t j0, const float4 *stg,
                                             const DeltaC &dcu, const DeltaC32 &dcu32,
                                             const float4 *tab, const double2 *tab64, double *zs,
                                             Acc<R, VARD, MIXED> &A)
{
    if constexpr (MIXED) {
        float px[R], py[R], pz[R];
#pragma unroll
        for (int r = 0; r < R; ++r) px[r] = py[r] = pz[r] = 0.0f;
#pragma unroll ZONE ? 1 : 2
        for (int j = 0; j < kCluster; ++j) {
            float sx32, sy32, sz32, gx32, gy32, gz32;
            src32<STAGE>(S, j0, stg, j, sx32, sy32, sz32, gx32, gy32, gz32);
            bool z64[R], any = false;
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const DeltaC32 &d32 = VARD ? A.dc32[VARD ? r : 0] : dcu32;
                near_pair32<ZONE>(A.tx32[r], A.ty32[r], A.tz32[r], sx32, sy32, sz32, gx32, gy32,
                                  gz32, d32, tab, px[r], py[r], pz[r]);
                if constexpr (ZONE) {
                    float dx, dy, dz;
                    z64[r] = diff32(A.tx32[r], A.ty32[r], A.tz32[r], sx32, sy32, sz32, dx, dy, dz) <
                             d32.cut2_64;
                    any = any || z64[r];
                }
            }
            if (ZONE && __builtin_amdgcn_ballot_w64(any)) {
                const double *e = S.d + (j0 + j) * 8;
                const double sx = e[0], sy = e[1], sz = e[2], gx = e[3], gy = e[4], gz = e[5];
                const int lane = threadIdx.x % kWave;
#pragma unroll
                for (int r = 0; r < R; ++r)
                    if (z64[r]) {
                        double *z = zs + r * 6 * kWave + lane;
                        double ax = z[3 * kWave], ay = z[4 * kWave], az = z[5 * kWave];
                        zone_pair64(z[0], z[kWave], z[2 * kWave], sx, sy, sz, gx, gy, gz,
                                    VARD ? A.dc[VARD ? r : 0] : dcu, ax, ay, az);
                        z[3 * kWave] = ax;
                        z[4 * kWave] = ay;
                        z[5 * kWave] = az;
                    }
            }
        }
#pragma unroll
        for (int r = 0; r < R; ++r) {
            two_sum_acc(px[r], A.hx[r], A.lx[r]);
            two_sum_acc(py[r], A.hy[r], A.ly[r]);
            two_sum_acc(pz[r], A.hz[r], A.lz[r]);
        }
    } else {
        DeltaC dcr[R];
#pragma unroll
        for (int r = 0; r < R; ++r) dcr[r] = VARD ? A.dc[VARD ? r : 0] : dcu;
        // unrolled twice, except at two or more targets a lane with one delta (their table rows
        // already fill the register file there)
#pragma unroll (R == 1 || VARD) ? 2 : 1
        for (int j = 0; j < kCluster; ++j) {
            const double *q = S.d + (j0 + j) * 8;
            const double sx = q[0], sy = q[1], sz = q[2], gx = q[3], gy = q[4], gz = q[5];
            near_pairs64<R>(A.tx, A.ty, A.tz, sx, sy, sz, gx, gy, gz, dcr, tab64, A.ax, A.ay, A.az);
        }
    }
}

// Lanes below this one whose bit is set in `mask`.
__device__ __forceinline__ uint32_t lanes_below(uint64_t mask)
{
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

// Classification of source cluster cl against the sphere `rec` of a target group (the plain
// sum), or by the FMM's box lists.
template <bool BOX>
__device__ __forceinline__ void classify(const PairArgs &a, const TBlockRec &rec,
                                         const double4 *__restrict__ sphere, int64_t cl,
                                         int64_t n_cl, int box, bool &far, bool &near)
{
    bool valid = cl < n_cl;
    if constexpr (BOX) {   // the FMM's box lists (wave-uniform mode)
        const int bs = a.fmm_box_src[valid ? cl : 0];
        const bool nb = a.fmm_near[(int64_t)box * a.fmm_k + bs] != 0;
        valid = valid && (a.fmm_mode == 1 ? nb : (a.fmm_mode == 2 ? !nb : bs == box));
    }
    far = valid && ((BOX && a.fmm_mode >= 2) || cluster_is_far(rec, sphere[valid ? cl : 0]));
    near = valid && !far;
}

// Far and near cluster counts of each target group, one wave per group.
template <int R, int G, bool BOX>
__global__ __launch_bounds__(4 * kWave) void k_counts(PairArgs a, const TBlockRec *__restrict__ recs,
                                                      const double4 *__restrict__ sphere,
                                                      uint2 *__restrict__ counts)
{
    const int n_groups = (a.n_tblocks + G - 1) / G;
    const int g = (int)blockIdx.x * 4 + (int)(threadIdx.x / kWave);
    if (g >= n_groups) return;
    const int lane = threadIdx.x % kWave;
    const int box = BOX ? a.fmm_box_tgt[(int64_t)g * G * R] : 0;
    const int64_t n_cl = a.s.np / kCluster;
    uint32_t nf = 0, nn = 0;
    for (int64_t c0 = 0; c0 < n_cl; c0 += kWave) {
        bool far, near;
        classify<BOX>(a, recs[g], sphere, c0 + lane, n_cl, box, far, near);
        nf += (uint32_t)__builtin_popcountll(__builtin_amdgcn_ballot_w64(far));
        nn += (uint32_t)__builtin_popcountll(__builtin_amdgcn_ballot_w64(near));
    }
    if (lane == 0) counts[g] = make_uint2(nf, nn);
}

// Work item (target block tb, way k).  The clusters are classified against the sphere `rec` of
// the block's group, scanned 64 at a time, one per lane; this way's share (mixed path: a range
// of far ranks and a range of near ranks, `nc` holding the group's far and near counts, and the
// scan ends with the ranges; FP64 path: the ranks congruent to k mod K) is picked with ballots
// and processed in ascending cluster order.  Every wave of a group walks the same clusters, so
// the group's waves share each source record in cache.
template <int R, bool VARD, bool MIXED, bool ZONE, bool STAGE, bool BOX>
__device__ __forceinline__ void pair_item(const PairArgs &a, const TBlockRec &rec,
                                          const TBlockRec &own, bool grouped, const Src &S,
                                          const double4 *__restrict__ sphere, const float4 *tab,
                                          const double2 *tab64, double *zs, float4 *stg,
                                          double *__restrict__ part, int tb, int k, int box, uint2 nc)
{
    const uint32_t K = (uint32_t)a.n_ways;
    const int lane = threadIdx.x % kWave;
    const int64_t t0 = (int64_t)tb * (kWave * R);
    const int64_t np_t = a.t.np;

    Acc<R, VARD, MIXED> A;
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int64_t i = t0 + r * kWave + lane;
        A.tx[r] = a.t.x[i];
        A.ty[r] = a.t.y[i];
        A.tz[r] = a.t.z[i];
        if constexpr (VARD) {
            A.dc[VARD ? r : 0] = make_delta(a.t.delta[i]);
            if constexpr (MIXED) A.dc32[VARD ? r : 0] = make_delta32(a.t.delta[i], a.rho64);
        }
        if constexpr (MIXED) {
            A.tx32[r] = a.t.x32[i];
            A.ty32[r] = a.t.y32[i];
            A.tz32[r] = a.t.z32[i];
            if constexpr (ZONE) {
                double *z = zs + r * 6 * kWave + lane;
                z[0] = A.tx[r];
                z[kWave] = A.ty[r];
                z[2 * kWave] = A.tz[r];
                z[3 * kWave] = z[4 * kWave] = z[5 * kWave] = 0.0;
            }
        }
        A.ax[r] = A.ay[r] = A.az[r] = 0.0;
        A.hx[r] = A.hy[r] = A.hz[r] = A.lx[r] = A.ly[r] = A.lz[r] = 0.0f;
    }
    const DeltaC dcu = make_delta(a.delta);
    const DeltaC32 dcu32 = make_delta32(a.delta, a.rho64);

    const int64_t n_cl = a.s.np / kCluster;
    // mixed path: this way's rank ranges (the products fit 64 bits: counts < 2^25, K <= 2^7)
    const uint32_t f_lo = (uint32_t)((uint64_t)k * nc.x / K), f_hi = (uint32_t)((uint64_t)(k + 1) * nc.x / K);
    const uint32_t n_lo = (uint32_t)((uint64_t)k * nc.y / K), n_hi = (uint32_t)((uint64_t)(k + 1) * nc.y / K);
    uint32_t rank_far = 0, rank_near = 0;
    for (int64_t c0 = 0; c0 < n_cl && (!MIXED || rank_far < f_hi || rank_near < n_hi); c0 += kWave) {
        bool far, near;
        classify<BOX>(a, rec, sphere, c0 + lane, n_cl, box, far, near);
        const uint64_t mf = __builtin_amdgcn_ballot_w64(far);
        const uint64_t mn = __builtin_amdgcn_ballot_w64(near);
        const uint32_t rf = rank_far + lanes_below(mf), rn = rank_near + lanes_below(mn);
        const bool take = MIXED ? (far ? (rf >= f_lo && rf < f_hi) : (near && rn >= n_lo && rn < n_hi))
                                : (far ? rf % K == (uint32_t)k : (near && rn % K == (uint32_t)k));
        const uint64_t mine = __builtin_amdgcn_ballot_w64(take);
        rank_far += (uint32_t)__builtin_popcountll(mf);
        rank_near += (uint32_t)__builtin_popcountll(mn);
        uint64_t m = mine;
        while (m) {
            const int b = __builtin_ctzll(m);
            m &= m - 1;
            const int64_t j0 = (c0 + b) * kCluster;
            if constexpr (STAGE) {
                // one record per lane; the wave reads back only what it wrote, after it, and a
                // wave's LDS operations complete in order
                const float4 *q = reinterpret_cast<const float4 *>(S.f + (j0 + lane) * 8);
                const float4 u = q[0], v = q[1];
                stg[2 * lane] = u;
                stg[2 * lane + 1] = v;
            }
            // near for the group, yet possibly far for this wave's own block
            if (((mf >> b) & 1) || (grouped && cluster_is_far(own, sphere[c0 + b])))
                far_cluster<R, VARD, MIXED, STAGE>(S, j0, stg, A);
            else
                near_cluster<R, VARD, MIXED, ZONE, STAGE>(S, j0, stg, dcu, dcu32, tab, tab64, zs, A);
        }
    }

    // The partial sums are read once, by the reduction: streaming stores keep them from
    // displacing the source records in L2.
    double *px = part + ((int64_t)k * 3 + 0) * np_t;
    double *py = part + ((int64_t)k * 3 + 1) * np_t;
    double *pz = part + ((int64_t)k * 3 + 2) * np_t;
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int64_t i = t0 + r * kWave + lane;
        if constexpr (MIXED) {
            double zx = 0.0, zy = 0.0, zz = 0.0;
            if constexpr (ZONE) {
                const double *z = zs + r * 6 * kWave + lane;
                zx = z[3 * kWave];
                zy = z[4 * kWave];
                zz = z[5 * kWave];
            }
            __builtin_nontemporal_store(zx + ((double)A.hx[r] + (double)A.lx[r]), px + i);
            __builtin_nontemporal_store(zy + ((double)A.hy[r] + (double)A.ly[r]), py + i);
            __builtin_nontemporal_store(zz + ((double)A.hz[r] + (double)A.lz[r]), pz + i);
        } else {
            __builtin_nontemporal_store(A.ax[r], px + i);
            __builtin_nontemporal_store(A.ay[r], py + i);
            __builtin_nontemporal_store(A.az[r], pz + i);
        }
    }
}

// Occupancy-sized grid of workgroups of G waves.  A workgroup pulls (group, way) items off the
// counter; wave w of the workgroup takes target block G * group + w.  Mixed path: items are
// way-major, so that the items in flight read the same slice of the source records; FP64 path:
// group-major.  ZONE (mixed path only): some near pairs are
// summed in double precision (rho64 > 0); without it the zone's code and LDS state are left out.
template <int R, bool VARD, bool MIXED, bool ZONE, int G, bool BOX>
__global__ __launch_bounds__(G * kWave) void k_pair(PairArgs a, const TBlockRec *__restrict__ recs,
                                                    const double *__restrict__ Sd,
                                                    const float *__restrict__ Sf,
                                                    const double4 *__restrict__ sphere,
                                                    double *__restrict__ part,
                                                    const uint2 *__restrict__ counts,
                                                    uint32_t *__restrict__ ctr)
{
    __shared__ uint32_t sh_item;
    // Single-precision smoothing table; the first barrier of the work loop publishes it.
    __shared__ float4 sh_tab[MIXED ? kTab32Rows : 1];
    if constexpr (MIXED) load_tab32(sh_tab);
    // FP64 path: the double-precision smoothing table, published by the same barrier.
    __shared__ double2 sh_tab64[MIXED ? 1 : kTab64Size2];
    if constexpr (!MIXED) load_tab64(sh_tab64);
    // Mixed path: the double-precision zone's per-target state, R * 6 * 64 doubles per wave.
    __shared__ double sh_zone[MIXED && ZONE ? G * R * 6 * kWave : 1];
    // Mixed path without the zone: each wave's copy of the cluster it works on, so that the
    // source loops take the source as a vector operand (an LDS broadcast) rather than a scalar
    // one, which halves the issue rate of single-precision instructions.
    constexpr bool STAGE = MIXED && !ZONE;
    __shared__ float4 sh_stage[STAGE ? G * 2 * kCluster : 1];
    const Src S{Sd, Sf};
    const uint32_t K = (uint32_t)a.n_ways;
    const int n_groups = (a.n_tblocks + G - 1) / G;
    const uint32_t n_items = (uint32_t)n_groups * K;
    const int w = threadIdx.x / kWave;
    for (;;) {
        if (threadIdx.x == 0) sh_item = atomicAdd(ctr, 1u);
        __syncthreads();
        const uint32_t item = sh_item;
        __syncthreads();
        if (item >= n_items) break;
        const int g = (int)(MIXED ? item % (uint32_t)n_groups : item / K);
        const int k = (int)(MIXED ? item / (uint32_t)n_groups : item % K);
        const int tb = g * G + w;
        const int box = BOX ? a.fmm_box_tgt[(int64_t)g * G * R] : 0;
        if (tb < a.n_tblocks)
            pair_item<R, VARD, MIXED, ZONE, STAGE, BOX>(
                a, recs[g], recs[G > 1 ? n_groups + tb : g], G > 1, S, sphere, sh_tab, sh_tab64,
                sh_zone + (MIXED && ZONE ? w * R * 6 * kWave : 0),
                sh_stage + (STAGE ? w * 2 * kCluster : 0), part, tb, k, box,
                MIXED ? counts[g] : make_uint2(0u, 0u));
    }
}

// Per target: the K way partials in way order.  A block of 4 waves serves 64 targets; wave w
// sums ways w, w + 4, ... and wave 0 adds the four sums in order.
__global__ __launch_bounds__(256) void k_reduce(const double *__restrict__ part, int n_ways,
                                                int64_t np, const int32_t *__restrict__ perm,
                                                double scale, double *__restrict__ ux,
                                                double *__restrict__ uy, double *__restrict__ uz)
{
    __shared__ double sh[4][3][kWave];
    const int lane = threadIdx.x % kWave, w = threadIdx.x / kWave;
    const int64_t p = (int64_t)blockIdx.x * kWave + lane;   // np is a multiple of 64
    double a = 0.0, b = 0.0, c = 0.0;
    for (int s = w; s < n_ways; s += 4) {
        a += __builtin_nontemporal_load(part + ((int64_t)s * 3 + 0) * np + p);
        b += __builtin_nontemporal_load(part + ((int64_t)s * 3 + 1) * np + p);
        c += __builtin_nontemporal_load(part + ((int64_t)s * 3 + 2) * np + p);
    }
    sh[w][0][lane] = a;
    sh[w][1][lane] = b;
    sh[w][2][lane] = c;
    __syncthreads();
    if (w != 0) return;
    const int32_t idx = perm[p];
    if (idx < 0) return;
    a = ((sh[0][0][lane] + sh[1][0][lane]) + sh[2][0][lane]) + sh[3][0][lane];
    b = ((sh[0][1][lane] + sh[1][1][lane]) + sh[2][1][lane]) + sh[3][1][lane];
    c = ((sh[0][2][lane] + sh[1][2][lane]) + sh[2][2][lane]) + sh[3][2][lane];
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

// Resident workgroups per CU of a kernel (queried once per kernel instance).
template <typename Kern>
int resident_blocks(Kern kernel, int threads)
{
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, (const void *)kernel, threads, 0) != hipSuccess ||
        nb < 1)
        nb = 1;
    return nb;
}

template <typename Kern>
unsigned work_grid(Kern kernel, int threads, int &cache, int n_cu, int64_t n_items)
{
    if (cache == 0) cache = resident_blocks(kernel, threads);
    const int64_t g = (int64_t)n_cu * cache;
    return (unsigned)(g < n_items ? g : n_items);
}

// Workgroup size (target blocks sharing one cluster stream): the mixed path gains from the
// shared scalar-cache lines; the FP64 path, whose loop is longer per source, runs one wave per
// workgroup.
template <bool MIXED>
constexpr int group_size() { return MIXED ? 4 : 1; }

template <int R>
hipError_t launch_r(const PairArgs &a, const PairPlan &p, bool mixed, bool vard, hipStream_t st,
                    const PairTiming *tm)
{
    static int occ[12] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
    const int G = mixed ? group_size<true>() : group_size<false>();
    const int n_groups = (p.n_tblocks + G - 1) / G;
    TBlockRec *rec = reinterpret_cast<TBlockRec *>(a.tblock_scratch);
    uint32_t *ctr = pair_counter(a.tblock_scratch, p.n_tblocks);
    uint2 *counts = reinterpret_cast<uint2 *>(reinterpret_cast<char *>(a.tblock_scratch) +
                                              (size_t)2 * p.n_tblocks * sizeof(TBlockRec));
    const SrcView &s = a.s;
    if (a.records_ready) {
        // written by the source gather
    } else if (mixed) {
        hipLaunchKernelGGL((k_tblock<R, group_size<true>()>), dim3(n_groups), dim3(group_size<true>() * kWave),
                           0, st, a, rec, 1, ctr);
    } else {
        hipLaunchKernelGGL((k_tblock<R, group_size<false>()>), dim3(n_groups), dim3(group_size<false>() * kWave),
                           0, st, a, rec, 0, ctr);
    }
    if (mixed) {
        const dim3 cg((unsigned)((n_groups + 3) / 4)), cb(4 * kWave);
        if (a.fmm_mode) {
            if constexpr (R <= 2)
                hipLaunchKernelGGL((k_counts<R, group_size<true>(), true>), cg, cb, 0, st, a, rec, s.sphere, counts);
        } else {
            hipLaunchKernelGGL((k_counts<R, group_size<true>(), false>), cg, cb, 0, st, a, rec, s.sphere, counts);
        }
    }
    if (tm && tm->e0) (void)hipEventRecord(tm->e0, st);
    const int64_t n_items = (int64_t)n_groups * p.n_ways;
    const bool zone = mixed && a.rho64 > 0.0;
#define SL_PAIR_LAUNCH(V, M, Z, B, SLOT)                                                            \
    hipLaunchKernelGGL((k_pair<R, V, M, Z, group_size<M>(), B>),                                     \
                       dim3(work_grid(k_pair<R, V, M, Z, group_size<M>(), B>, group_size<M>() * kWave,\
                                      occ[SLOT], p.n_cu, n_items)),                                  \
                       dim3(group_size<M>() * kWave), 0, st, a, rec, s.d, s.f32, s.sphere, a.part, counts, ctr)
    if (a.fmm_mode) {
        // The FMM's cluster lists: instances of their own, so that the plain sum's kernels carry
        // none of the list code (two targets per lane at most).
        if constexpr (R <= 2) {
            if (vard) {
                if (zone) SL_PAIR_LAUNCH(true, true, true, true, 9);
                else if (mixed) SL_PAIR_LAUNCH(true, true, false, true, 11);
                else SL_PAIR_LAUNCH(true, false, false, true, 7);
            } else {
                if (zone) SL_PAIR_LAUNCH(false, true, true, true, 8);
                else if (mixed) SL_PAIR_LAUNCH(false, true, false, true, 10);
                else SL_PAIR_LAUNCH(false, false, false, true, 6);
            }
        } else {
            return hipErrorInvalidValue;
        }
    } else if (vard) {
        if (zone) SL_PAIR_LAUNCH(true, true, true, false, 3);
        else if (mixed) SL_PAIR_LAUNCH(true, true, false, false, 5);
        else SL_PAIR_LAUNCH(true, false, false, false, 1);
    } else {
        if (zone) SL_PAIR_LAUNCH(false, true, true, false, 2);
        else if (mixed) SL_PAIR_LAUNCH(false, true, false, false, 4);
        else SL_PAIR_LAUNCH(false, false, false, false, 0);
    }
#undef SL_PAIR_LAUNCH
    if (tm && tm->e1) (void)hipEventRecord(tm->e1, st);
    return hipGetLastError();
}

}  // namespace

// Target-group and target-block records (at most 2 n_tblocks), the groups' cluster counts (at
// most n_tblocks), then 256 bytes holding the work counter.
size_t tblock_scratch_bytes(int n_tblocks)
{
    return (size_t)2 * n_tblocks * sizeof(TBlockRec) + (size_t)round_up((int64_t)n_tblocks * 8, 256) + 256;
}

int pair_group_size(bool mixed) { return mixed ? group_size<true>() : group_size<false>(); }

uint32_t *pair_counter(void *tblock_scratch, int n_tblocks)
{
    return reinterpret_cast<uint32_t *>(reinterpret_cast<char *>(tblock_scratch) +
                                        tblock_scratch_bytes(n_tblocks) - 256);
}

PairPlan plan_pairs(int64_t np_src, int64_t np_tgt, int R, int waves_wanted, bool mixed)
{
    PairPlan p;
    p.R = R;
    p.n_tblocks = (int)(np_tgt / (kWave * R));
    const int64_t n_cl = np_src / kCluster;
    const int64_t cap = mixed ? kMaxWaysMixed : kMaxWays;
    int64_t K = (waves_wanted + p.n_tblocks - 1) / p.n_tblocks;
    K = K < 1 ? 1 : (K > cap ? cap : K);
    K = K > n_cl ? n_cl : K;
    p.n_ways = (int)K;
    p.n_cu = 0;
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

hipError_t launch_reduce(const double *part, int n_ways, int64_t np, const int32_t *perm,
                         double scale, double *ux, double *uy, double *uz, hipStream_t st)
{
    hipLaunchKernelGGL(k_reduce, dim3((unsigned)(np / kWave)), dim3(256), 0, st, part, n_ways, np,
                       perm, scale, ux, uy, uz);
    return hipGetLastError();
}

hipError_t launch_fill_zero(double *ux, double *uy, double *uz, int64_t n, hipStream_t st)
{
    hipLaunchKernelGGL(k_fill_zero, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, ux, uy,
                       uz, n);
    return hipGetLastError();
}

}  // namespace sl
