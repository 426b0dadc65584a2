// sl_fmm.hip -- single-level kernel-independent FMM of the single layer (Sec. 5, "Fast multipole
// method based acceleration").  The paper's steps:
//   1. k-means clustering of the points into k clusters (the paper takes k = 100);
//   2. per cluster, a cube (the equivalent surface) carrying equivalent sources on a regular grid
//      of its boundary and a larger cube (the check surface); the equivalent densities reproduce on
//      the check surface the potential of the cluster's own points;
//   3. the sum over points of neighbouring clusters directly, over the other clusters from their
//      equivalent sources.
//
// On the device:
//   * k-means: Lloyd iterations, one assignment kernel and one update kernel each, all launched up
//     front (a device flag turns the remaining ones into no-ops once no label changes).  A point
//     joins the nearest centroid (squared distance ((dx dx + dy dy) + dz dz) with round-to-nearest
//     products and sums, ties to the lower index); centroid sums are exact 64-bit integer sums of
//     the coordinates quantized to 2^-24 of the extent, so the clustering does not depend on the
//     order in which the atomics land;
//   * the boxes' extents (integer atomics on order-preserving encodings of the coordinates) come
//     back to the host, which forms the cubes, the near/far lists and the padded layout: every box
//     holds a multiple of 256 points, so whole target groups and source clusters belong to one box;
//   * the points are scattered box by box (stable: input order within a box) into the pair
//     kernel's records;
//   * check potentials (pair kernel, plain Stokeslet, each box's check points against its own
//     points), equivalent densities phi = a M_unit v (M_unit: the Tikhonov least-squares operator
//     of the unit box, built on the host once per grid size and kept by the context), and the
//     equivalent sources' records;
//   * near field (pair kernel over near boxes, the regularized kernel) and far field (pair kernel
//     over the equivalent sources of far boxes, plain Stokeslet) into one set of per-way partial
//     sums, added in a fixed order by the reduction.
// Constants (the paper gives no values): equivalent and check surfaces at 1.05 and 2.95 times the
// cluster's half width, far boxes outside the cube of 3 half widths around a cluster and at least
// 6.9 delta away (where s1 = s2 = 1 in double precision, so the far field is the plain Stokeslet),
// Tikhonov weight 1e-8 of the largest squared column norm.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <string>
#include <vector>

#include "sl_internal.h"

namespace sl {

namespace {

constexpr double kAlphaEq = 1.05;
constexpr double kAlphaCheck = 2.95;
constexpr double kAlphaFar = 3.0;
constexpr double kTikhonov = 1e-8;
constexpr int kBoxPad = 256;          // points of a box: a multiple of one target group
constexpr int kMaxBoxes = 1024;
constexpr int kQuantBits = 24;

// ---------------------------------------------------------------------------------------------
// Order-preserving 64-bit encoding of doubles (for integer atomic min / max).
__device__ __forceinline__ uint64_t enc(double v)
{
    const uint64_t u = (uint64_t)__double_as_longlong(v);
    return (u >> 63) ? ~u : (u | (1ull << 63));
}
double dec(uint64_t e)
{
    const uint64_t u = (e >> 63) ? (e & ~(1ull << 63)) : ~e;
    double v;
    memcpy(&v, &u, 8);
    return v;
}

struct KmState {
    double lo[3];
    double scale;          // 2^(24 - e), 2^e >= the largest axis extent
    uint32_t done;         // no label changed in the last assignment
    uint32_t changed;      // labels changed by the current assignment
    uint32_t iterations;   // assignments made
    uint32_t pad;
};

// Bounding box of all points (one workgroup, exact min / max) and the quantization scale.
__global__ __launch_bounds__(1024) void k_km_box(const double *__restrict__ x, const double *__restrict__ y,
                                                 const double *__restrict__ z, int64_t n,
                                                 KmState *__restrict__ st, double *__restrict__ box)
{
    double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    for (int64_t i = threadIdx.x; i < n; i += blockDim.x) {
        const double p[3] = {x[i], y[i], z[i]};
        for (int c = 0; c < 3; ++c) { lo[c] = fmin(lo[c], p[c]); hi[c] = fmax(hi[c], p[c]); }
    }
    __shared__ double red[6][16];
    const int w = threadIdx.x / kWave, lane = threadIdx.x % kWave;
    for (int c = 0; c < 3; ++c) {
        const double l = wave_min(lo[c]), h = wave_max(hi[c]);
        if (lane == 0) { red[c][w] = l; red[3 + c][w] = h; }
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double b[6];
        for (int c = 0; c < 6; ++c) {
            double v = red[c][0];
            for (int j = 1; j < (int)(blockDim.x / kWave); ++j) v = c < 3 ? fmin(v, red[c][j]) : fmax(v, red[c][j]);
            b[c] = v;
        }
        double ext = 0.0;
        for (int c = 0; c < 3; ++c) {
            box[c] = b[c];
            box[3 + c] = b[3 + c];
            st->lo[c] = b[c];
            ext = fmax(ext, b[3 + c] - b[c]);
        }
        int e = 0;
        if (ext > 0.0) (void)frexp(ext, &e);     // ext < 2^e
        st->scale = ldexp(1.0, kQuantBits - e);
        st->done = 0;
        st->changed = 0;
        st->iterations = 0;
    }
}

// Initial centroids: the points at indices floor(j n / k); no label yet.
__global__ __launch_bounds__(256) void k_km_init(const double *__restrict__ x, const double *__restrict__ y,
                                                 const double *__restrict__ z, int64_t n, int k,
                                                 double *__restrict__ C, int32_t *__restrict__ labels,
                                                 unsigned long long *__restrict__ sums)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < k) {
        const int64_t p = (i * n) / k;
        C[3 * i] = x[p];
        C[3 * i + 1] = y[p];
        C[3 * i + 2] = z[p];
        for (int c = 0; c < 4; ++c) sums[4 * i + c] = 0ull;
    }
    if (i < n) labels[i] = -1;
}

// One assignment: nearest centroid per point, labels changed, exact per-cluster coordinate sums
// (workgroup sums in LDS, then one global atomic per cluster and workgroup).
__global__ __launch_bounds__(256) void k_km_assign(const double *__restrict__ x, const double *__restrict__ y,
                                                   const double *__restrict__ z, int64_t n, int k,
                                                   const double *__restrict__ C, int32_t *__restrict__ labels,
                                                   KmState *__restrict__ st,
                                                   unsigned long long *__restrict__ sums)
{
    if (st->done) return;
    extern __shared__ unsigned long long lds[];        // 4 k sums, then 3 k centroid coordinates
    unsigned long long *ss = lds;
    double *sc = reinterpret_cast<double *>(lds + 4 * k);
    for (int j = threadIdx.x; j < 3 * k; j += blockDim.x) sc[j] = C[j];
    for (int j = threadIdx.x; j < 4 * k; j += blockDim.x) ss[j] = 0ull;
    __syncthreads();
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    bool changed = false;
    if (i < n) {
        const double px = x[i], py = y[i], pz = z[i];
        int best = 0;
        double bd = INFINITY;
        for (int j = 0; j < k; ++j) {
            const double dx = px - sc[3 * j], dy = py - sc[3 * j + 1], dz = pz - sc[3 * j + 2];
            const double d2 = __dadd_rn(__dadd_rn(__dmul_rn(dx, dx), __dmul_rn(dy, dy)), __dmul_rn(dz, dz));
            if (d2 < bd) { bd = d2; best = j; }
        }
        changed = labels[i] != best;
        labels[i] = best;
        const double s = st->scale;
        const long long qx = (long long)rint(__dmul_rn(px - st->lo[0], s));
        const long long qy = (long long)rint(__dmul_rn(py - st->lo[1], s));
        const long long qz = (long long)rint(__dmul_rn(pz - st->lo[2], s));
        atomicAdd(&ss[4 * best], (unsigned long long)qx);
        atomicAdd(&ss[4 * best + 1], (unsigned long long)qy);
        atomicAdd(&ss[4 * best + 2], (unsigned long long)qz);
        atomicAdd(&ss[4 * best + 3], 1ull);
    }
    const uint64_t m = __builtin_amdgcn_ballot_w64(changed);
    if (threadIdx.x % kWave == 0 && m) atomicAdd(&st->changed, (uint32_t)__builtin_popcountll(m));
    __syncthreads();
    for (int j = threadIdx.x; j < 4 * k; j += blockDim.x)
        if (ss[j]) atomicAdd(&sums[j], ss[j]);
}

// Centroids from the sums (an empty cluster keeps its centroid), or the end of the iteration when
// no label changed.  One workgroup; clears the sums for the next assignment.
__global__ __launch_bounds__(1024) void k_km_update(int k, double *__restrict__ C, KmState *__restrict__ st,
                                                   unsigned long long *__restrict__ sums)
{
    if (st->done) return;
    __shared__ uint32_t changed;
    if (threadIdx.x == 0) changed = st->changed;
    __syncthreads();
    if (threadIdx.x == 0) {
        st->iterations += 1;
        st->changed = 0;
        if (changed == 0) st->done = 1;
    }
    for (int j = threadIdx.x; j < k; j += blockDim.x) {
        const unsigned long long cnt = sums[4 * j + 3];
        if (changed != 0 && cnt > 0) {
            for (int c = 0; c < 3; ++c) {
                const double q = (double)(long long)sums[4 * j + c];
                C[3 * j + c] = st->lo[c] + (q / (double)cnt) / st->scale;
            }
        }
        for (int c = 0; c < 4; ++c) sums[4 * j + c] = 0ull;
    }
}

// Per-cluster extents (encoded min / max), point counts and largest delta.
__global__ __launch_bounds__(256) void k_box_init(int k, unsigned long long *__restrict__ ext,
                                                  unsigned long long *__restrict__ dmax,
                                                  unsigned int *__restrict__ cnt)
{
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= k) return;
    for (int c = 0; c < 3; ++c) {
        ext[6 * j + c] = ~0ull;
        ext[6 * j + 3 + c] = 0ull;
    }
    dmax[j] = 0ull;
    cnt[j] = 0u;
}

__global__ __launch_bounds__(256) void k_box_extent(const double *__restrict__ x, const double *__restrict__ y,
                                                    const double *__restrict__ z, const double *__restrict__ dt,
                                                    double delta, int64_t n, const int32_t *__restrict__ labels,
                                                    unsigned long long *__restrict__ ext,
                                                    unsigned long long *__restrict__ dmax,
                                                    unsigned int *__restrict__ cnt)
{
    // per wave and label, the extents reduced across the wave first (exact: min / max), then
    // one set of atomics
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int lane = threadIdx.x % kWave;
    const int lab = i < n ? labels[i] : -1;
    double p[3] = {0.0, 0.0, 0.0}, dl = 0.0;
    if (i < n) {
        p[0] = x[i]; p[1] = y[i]; p[2] = z[i];
        dl = dt ? dt[i] : delta;
    }
    for (uint64_t left = __builtin_amdgcn_ballot_w64(lab >= 0); left;) {
        const int first = __builtin_ctzll(left);
        const int j = __shfl(lab, first, kWave);
        const bool mine = lab == j;
        const uint64_t mask = __builtin_amdgcn_ballot_w64(mine);
        left &= ~mask;
        double lo[3], hi[3];
        for (int c = 0; c < 3; ++c) {
            lo[c] = wave_min(mine ? p[c] : INFINITY);
            hi[c] = wave_max(mine ? p[c] : -INFINITY);
        }
        const double dm = wave_max(mine ? dl : -INFINITY);
        if (lane == first) {
            for (int c = 0; c < 3; ++c) {
                atomicMin(&ext[6 * j + c], (unsigned long long)enc(lo[c]));
                atomicMax(&ext[6 * j + 3 + c], (unsigned long long)enc(hi[c]));
            }
            atomicMax(&dmax[j], (unsigned long long)enc(dm));
            atomicAdd(&cnt[j], (unsigned int)__builtin_popcountll(mask));
        }
    }
}

// Stable box order: rank of each point among the earlier points of its box within its wave, and
// per wave the count of each box (wcnt[wave][box], cleared first).
__global__ __launch_bounds__(256) void k_rank_in_wave(const int32_t *__restrict__ labels, int64_t n, int k,
                                                      uint32_t *__restrict__ rank, uint32_t *__restrict__ wcnt)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int lane = threadIdx.x % kWave;
    const int64_t wave = i / kWave;
    const int lab = i < n ? labels[i] : -1;
    uint32_t r = 0, total = 0;
    for (int l = 0; l < kWave; ++l) {
        const int o = __shfl(lab, l, kWave);
        if (o == lab) {
            total += 1;
            if (l < lane) r += 1;
        }
    }
    if (i < n) {
        rank[i] = r;
        if (r + 1 == total) wcnt[wave * k + lab] = total;   // the last of its box in the wave
    }
}

// Per box, the exclusive prefix of its wave counts (one wave per box).
__global__ __launch_bounds__(kWave) void k_scan_waves(int64_t n_waves, int k, uint32_t *__restrict__ wcnt)
{
    const int j = blockIdx.x, lane = threadIdx.x;
    uint32_t carry = 0;
    for (int64_t w0 = 0; w0 < n_waves; w0 += kWave) {
        const int64_t w = w0 + lane;
        const uint32_t v = w < n_waves ? wcnt[w * k + j] : 0u;
        uint32_t s = v;   // inclusive scan across the wave
        for (int o = 1; o < kWave; o <<= 1) {
            const uint32_t t = __shfl_up(s, o, kWave);
            if (lane >= o) s += t;
        }
        if (w < n_waves) wcnt[w * k + j] = carry + s - v;
        carry += __shfl(s, kWave - 1, kWave);
    }
}

struct SortedOut {
    double *x, *y, *z;        // structure-of-arrays positions (targets)
    float *x32, *y32, *z32;   // single-precision copies relative to the box centre (mixed)
    double *d;                // [np][8] FP64 source records
    float *f32;               // [np][8] FP32 source records (mixed)
    double *delta;            // per-target delta (nullptr: none)
    int32_t *perm;            // sorted position -> input index (-1: padding)
};

__device__ __forceinline__ void put_point(const SortedOut &o, int64_t p, double px, double py, double pz,
                                          double gx, double gy, double gz, const double *centre, double dlt,
                                          int32_t idx)
{
    o.x[p] = px; o.y[p] = py; o.z[p] = pz;
    double *r = o.d + p * 8;
    r[0] = px; r[1] = py; r[2] = pz; r[3] = gx; r[4] = gy; r[5] = gz; r[6] = 0.0; r[7] = 0.0;
    if (o.f32) {
        const float fx = (float)(px - centre[0]), fy = (float)(py - centre[1]), fz = (float)(pz - centre[2]);
        o.x32[p] = fx; o.y32[p] = fy; o.z32[p] = fz;
        float *q = o.f32 + p * 8;
        q[0] = fx; q[1] = fy; q[2] = fz; q[3] = (float)gx; q[4] = (float)gy; q[5] = (float)gz;
        q[6] = 0.0f; q[7] = 0.0f;
    }
    if (o.delta) o.delta[p] = dlt;
    o.perm[p] = idx;
}

__global__ __launch_bounds__(256) void k_scatter_boxes(const double *__restrict__ x, const double *__restrict__ y,
                                                       const double *__restrict__ z, const double *__restrict__ w,
                                                       const double *__restrict__ fx, const double *__restrict__ fy,
                                                       const double *__restrict__ fz, const double *__restrict__ dt,
                                                       int64_t n, int k, const int32_t *__restrict__ labels,
                                                       const uint32_t *__restrict__ rank,
                                                       const uint32_t *__restrict__ wbase,
                                                       const int64_t *__restrict__ off,
                                                       const double *__restrict__ centre, SortedOut o)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int j = labels[i];
    const int64_t p = off[j] + wbase[(i / kWave) * k + j] + rank[i];
    const double wi = w[i];
    put_point(o, p, x[i], y[i], z[i], wi * fx[i], wi * fy[i], wi * fz[i], centre, dt ? dt[i] : 0.0, (int32_t)i);
}

// Padding of each box to a multiple of kBoxPad: the box centre, zero density, delta of the box.
__global__ __launch_bounds__(256) void k_pad_boxes(int k, const int64_t *__restrict__ off,
                                                   const int64_t *__restrict__ cnt,
                                                   const double *__restrict__ boxc,
                                                   const double *__restrict__ bdelta,
                                                   const double *__restrict__ centre, SortedOut o)
{
    const int j = blockIdx.x, t = threadIdx.x;
    const int64_t p = off[j] + cnt[j] + t;
    if (p >= off[j + 1]) return;
    put_point(o, p, boxc[4 * j], boxc[4 * j + 1], boxc[4 * j + 2], 0.0, 0.0, 0.0, centre, bdelta[j], -1);
}

// Bounding sphere of each cluster of 64 records (centre of the box, farthest member, margin 2^-40).
__global__ __launch_bounds__(kWave) void k_cluster_spheres(const double *__restrict__ d, double4 *__restrict__ sph)
{
    const int64_t c = blockIdx.x;
    const double *r = d + (c * kCluster + threadIdx.x) * 8;
    const double px = r[0], py = r[1], pz = r[2];
    const double cx = 0.5 * (wave_min(px) + wave_max(px));
    const double cy = 0.5 * (wave_min(py) + wave_max(py));
    const double cz = 0.5 * (wave_min(pz) + wave_max(pz));
    const double dx = px - cx, dy = py - cy, dz = pz - cz;
    const double rr = wave_max(fma(dx, dx, fma(dy, dy, __dmul_rn(dz, dz))));
    if (threadIdx.x == 0) sph[c] = make_double4(cx, cy, cz, sqrt(rr) * (1.0 + 0x1p-40));
}

// Equivalent densities phi_j = a_j M v_j: M is (3 ne) x (3 nc), v_j = (vx, vy, vz) of box j's check
// points (component-major), phi into the equivalent sources' records (component-major rows).
__global__ __launch_bounds__(256) void k_equiv_density(int k, int ne, int nc, const double *__restrict__ M,
                                                       const double *__restrict__ vx, const double *__restrict__ vy,
                                                       const double *__restrict__ vz,
                                                       const double *__restrict__ boxc, int pe,
                                                       double *__restrict__ erec, float *__restrict__ erec32)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;   // (box, row)
    if (t >= (int64_t)k * 3 * ne) return;
    const int j = (int)(t / (3 * ne)), row = (int)(t % (3 * ne));
    const double *m = M + (int64_t)row * 3 * nc;
    const double *v[3] = {vx + (int64_t)j * nc, vy + (int64_t)j * nc, vz + (int64_t)j * nc};
    double s = 0.0;
    for (int c = 0; c < 3; ++c)
        for (int i = 0; i < nc; ++i) s = fma(m[c * nc + i], v[c][i], s);
    const double phi = boxc[4 * j + 3] * s;
    const int comp = row / ne, e = row % ne;
    const int64_t p = (int64_t)j * pe + e;
    erec[p * 8 + 3 + comp] = phi;
    if (erec32) erec32[p * 8 + 3 + comp] = (float)phi;
}

// Positions of equivalent-source records (from host-computed positions), zero density and
// zero padding; FP32 copies relative to the centre.
__global__ __launch_bounds__(256) void k_equiv_records(int64_t n, const double *__restrict__ pos,
                                                       const double *__restrict__ centre,
                                                       double *__restrict__ erec, float *__restrict__ erec32)
{
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n) return;
    const double px = pos[3 * p], py = pos[3 * p + 1], pz = pos[3 * p + 2];
    double *r = erec + p * 8;
    r[0] = px; r[1] = py; r[2] = pz; r[3] = r[4] = r[5] = r[6] = r[7] = 0.0;
    if (erec32) {
        float *q = erec32 + p * 8;
        q[0] = (float)(px - centre[0]); q[1] = (float)(py - centre[1]); q[2] = (float)(pz - centre[2]);
        q[3] = q[4] = q[5] = q[6] = q[7] = 0.0f;
    }
}

__global__ __launch_bounds__(256) void k_copy_labels(const int32_t *__restrict__ a, int64_t n, int32_t *__restrict__ b)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) b[i] = a[i];
}

unsigned blocks_of(int64_t n, int t) { return (unsigned)((n + t - 1) / t); }

// ---------------------------------------------------------------------------------------------
// Host: the unit box's operator.
// The lattice points on the boundary of [-1, 1]^3, p per edge, lexicographic.
std::vector<double> cube_points(int p)
{
    std::vector<double> g(p), pts;
    for (int i = 0; i < p; ++i) g[i] = -1.0 + 2.0 * i / (p - 1);
    for (int i = 0; i < p; ++i)
        for (int j = 0; j < p; ++j)
            for (int l = 0; l < p; ++l)
                if (i == 0 || i == p - 1 || j == 0 || j == p - 1 || l == 0 || l == p - 1) {
                    pts.push_back(g[i]);
                    pts.push_back(g[j]);
                    pts.push_back(g[l]);
                }
    return pts;
}

// M = argmin |K M - I|^2 + lambda |M|^2 column by column, i.e. the least-squares solution of
// [K; sqrt(lambda) I] M = [I; 0], by Householder QR of the stacked matrix (column-major).
// K (m x n) is the plain Stokeslet from the n / 3 equivalent to the m / 3 check points of the
// unit box; the result is n x m, row-major.
std::vector<double> unit_operator(int p)
{
    const std::vector<double> E = cube_points(p);
    const int ne = (int)E.size() / 3, m = 3 * ne, n = 3 * ne, rows = m + n;
    std::vector<double> A((size_t)rows * n, 0.0);          // column-major
    double colmax = 0.0;
    for (int b = 0; b < 3; ++b)
        for (int j = 0; j < ne; ++j) {
            double *col = &A[(size_t)(b * ne + j) * rows];
            double nrm = 0.0;
            for (int a = 0; a < 3; ++a)
                for (int i = 0; i < ne; ++i) {
                    double d[3];
                    for (int c = 0; c < 3; ++c) d[c] = kAlphaCheck * E[3 * i + c] - kAlphaEq * E[3 * j + c];
                    const double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
                    const double r = sqrt(r2);
                    const double v = (a == b ? 1.0 / r : 0.0) + d[a] * d[b] / (r2 * r);
                    col[a * ne + i] = v;
                    nrm += v * v;
                }
            colmax = std::max(colmax, nrm);
        }
    const double sl = sqrt(kTikhonov * colmax);
    for (int j = 0; j < n; ++j) A[(size_t)j * rows + m + j] = sl;
    std::vector<double> B((size_t)rows * m, 0.0);           // [I; 0], column-major
    for (int i = 0; i < m; ++i) B[(size_t)i * rows + i] = 1.0;
    std::vector<double> v(rows);
    for (int j = 0; j < n; ++j) {
        double *aj = &A[(size_t)j * rows];
        double nrm = 0.0;
        for (int i = j; i < rows; ++i) nrm += aj[i] * aj[i];
        nrm = sqrt(nrm);
        const double alpha = aj[j] > 0.0 ? -nrm : nrm;
        for (int i = j; i < rows; ++i) v[i] = aj[i];
        v[j] -= alpha;
        double vv = 0.0;
        for (int i = j; i < rows; ++i) vv += v[i] * v[i];
        if (vv == 0.0) continue;
        const double beta = 2.0 / vv;
        auto reflect = [&](double *col) {
            double s = 0.0;
            for (int i = j; i < rows; ++i) s += v[i] * col[i];
            s *= beta;
            for (int i = j; i < rows; ++i) col[i] -= s * v[i];
        };
        for (int c = j; c < n; ++c) reflect(&A[(size_t)c * rows]);
        for (int c = 0; c < m; ++c) reflect(&B[(size_t)c * rows]);
    }
    // back substitution R M = B[0:n, :]
    std::vector<double> M((size_t)n * m);
    for (int c = 0; c < m; ++c) {
        const double *bc = &B[(size_t)c * rows];
        for (int i = n - 1; i >= 0; --i) {
            double s = bc[i];
            for (int l = i + 1; l < n; ++l) s -= A[(size_t)l * rows + i] * M[(size_t)l * m + c];
            M[(size_t)i * m + c] = s / A[(size_t)i * rows + i];
        }
    }
    return M;
}

}  // namespace

}  // namespace sl

using namespace sl;

extern "C" {

sl_status sl_eval_fmm(sl_ctx *ctx, sl_precision prec, int64_t n, const double *x, const double *y,
                      const double *z, const double *w, const double *fx, const double *fy,
                      const double *fz, double delta, const double *delta_tgt, double mu, int k,
                      int p_edge, int max_iter, double *ux, double *uy, double *uz, int32_t *labels_out,
                      void *stream)
{
    const char *who = "sl_eval_fmm: ";
    if (!ctx) return fail(SL_EINVAL, "sl_eval_fmm: ctx is NULL");
    if (prec != SL_FP64 && prec != SL_MIXED) return fail(SL_EINVAL, std::string(who) + "unknown precision");
    if (n < 1 || n > ((int64_t)1 << 28)) return fail(SL_EINVAL, std::string(who) + "n must be in 1..2^28");
    if (k < 1 || k > kMaxBoxes || k > n) return fail(SL_EINVAL, std::string(who) + "need 1 <= k <= min(n, 1024)");
    if (p_edge < 3 || p_edge > 12) return fail(SL_EINVAL, std::string(who) + "need 3 <= p <= 12 points per cube edge");
    if (max_iter < 1 || max_iter > 10000) return fail(SL_EINVAL, std::string(who) + "need 1 <= max_iter <= 10000");
    if (!(isfinite(mu) && mu > 0.0)) return fail(SL_EINVAL, std::string(who) + "mu must be finite and > 0");
    if (!delta_tgt && !(isfinite(delta) && delta > 0.0))
        return fail(SL_EINVAL, std::string(who) + "delta must be finite and > 0");
    if (!x || !y || !z || !w || !fx || !fy || !fz || !ux || !uy || !uz)
        return fail(SL_EINVAL, std::string(who) + "NULL array");
    {
        const char *outs[3] = {(const char *)ux, (const char *)uy, (const char *)uz};
        const char *ins[8] = {(const char *)x, (const char *)y, (const char *)z, (const char *)w,
                              (const char *)fx, (const char *)fy, (const char *)fz, (const char *)delta_tgt};
        const int64_t b = n * 8;
        for (int a = 0; a < 3; ++a) {
            for (int c = a + 1; c < 3; ++c)
                if (outs[a] < outs[c] + b && outs[c] < outs[a] + b)
                    return fail(SL_EINVAL, std::string(who) + "outputs overlap");
            for (const char *in : ins)
                if (in && outs[a] < in + b && in < outs[a] + b)
                    return fail(SL_EINVAL, std::string(who) + "output aliases an input");
        }
    }
    struct Guard {
        int prev = -1;
        ~Guard() { if (prev >= 0) (void)hipSetDevice(prev); }
    } guard;
    if (hipGetDevice(&guard.prev) != hipSuccess) guard.prev = -1;
    if (hipSetDevice(ctx->device) != hipSuccess) return fail(SL_EHIP, std::string(who) + "hipSetDevice failed");
    const hipStream_t st = (hipStream_t)stream;
    const bool mixed = prec == SL_MIXED;
    const bool vard = delta_tgt != nullptr;

    // unit-box operator for this grid (host QR once per p, kept by the context)
    double *Mdev = nullptr;
    {
        std::lock_guard<std::mutex> l(ctx->mu);
        auto it = ctx->fmm_ops.find(p_edge);
        if (it != ctx->fmm_ops.end()) {
            Mdev = it->second;
        } else {
            const std::vector<double> M = unit_operator(p_edge);
            hipError_t e = hipMalloc(&Mdev, M.size() * sizeof(double));
            if (e == hipSuccess) e = hipMemcpy(Mdev, M.data(), M.size() * sizeof(double), hipMemcpyHostToDevice);
            if (e != hipSuccess) {
                if (Mdev) (void)hipFree(Mdev);
                return hip_fail(e, "sl_eval_fmm: unit operator");
            }
            ctx->fmm_ops[p_edge] = Mdev;
        }
    }
    const std::vector<double> E = cube_points(p_edge);
    const int ne = (int)E.size() / 3;

    // ---- stage 1: k-means and box extents (workspace A) -----------------------------------
    const int64_t n_waves = (n + kWave - 1) / kWave;
    size_t off = 0;
    auto take = [&](size_t bytes) { size_t o = off; off += (size_t)round_up((int64_t)bytes, 256); return o; };
    const size_t o_state = take(sizeof(KmState)), o_box = take(6 * 8), o_C = take((size_t)3 * k * 8);
    const size_t o_sums = take((size_t)4 * k * 8), o_lab = take((size_t)n * 4), o_ext = take((size_t)6 * k * 8);
    const size_t o_dmax = take((size_t)k * 8), o_cnt = take((size_t)k * 4), o_rank = take((size_t)n * 4);
    const size_t o_wcnt = take((size_t)n_waves * k * 4);
    char *A = nullptr;
    hipError_t e = ws_alloc(ctx, (void **)&A, off, st);
    if (e != hipSuccess) return hip_fail(e, "sl_eval_fmm: workspace");
    KmState *kst = (KmState *)(A + o_state);
    double *gbox = (double *)(A + o_box), *C = (double *)(A + o_C);
    unsigned long long *sums = (unsigned long long *)(A + o_sums);
    int32_t *labels = (int32_t *)(A + o_lab);
    unsigned long long *ext = (unsigned long long *)(A + o_ext), *dmax = (unsigned long long *)(A + o_dmax);
    unsigned int *cnt = (unsigned int *)(A + o_cnt);
    uint32_t *rank = (uint32_t *)(A + o_rank), *wcnt = (uint32_t *)(A + o_wcnt);
    char *B = nullptr;   // stage-2 workspace
    auto cleanup = [&](hipError_t err, const char *what) -> sl_status {
        if (B) (void)hipFreeAsync(B, st);
        if (A) (void)hipFreeAsync(A, st);
        return hip_fail(err, what);
    };

    hipLaunchKernelGGL(k_km_box, dim3(1), dim3(1024), 0, st, x, y, z, n, kst, gbox);
    hipLaunchKernelGGL(k_km_init, dim3(blocks_of(std::max<int64_t>(n, k), 256)), dim3(256), 0, st, x, y, z, n, k, C,
                       labels, sums);
    for (int it = 0; it < max_iter; ++it) {
        hipLaunchKernelGGL(k_km_assign, dim3(blocks_of(n, 256)), dim3(256), (size_t)7 * k * 8, st, x, y, z, n, k, C,
                           labels, kst, sums);
        hipLaunchKernelGGL(k_km_update, dim3(1), dim3(1024), 0, st, k, C, kst, sums);
    }
    hipLaunchKernelGGL(k_box_init, dim3(blocks_of(k, 256)), dim3(256), 0, st, k, ext, dmax, cnt);
    hipLaunchKernelGGL(k_box_extent, dim3(blocks_of(n, 256)), dim3(256), 0, st, x, y, z, delta_tgt, delta, n, labels,
                       ext, dmax, cnt);
    e = hipMemsetAsync(wcnt, 0, (size_t)n_waves * k * 4, st);
    if (e != hipSuccess) return cleanup(e, "sl_eval_fmm: clear");
    hipLaunchKernelGGL(k_rank_in_wave, dim3(blocks_of(n, 256)), dim3(256), 0, st, labels, n, k, rank, wcnt);
    hipLaunchKernelGGL(k_scan_waves, dim3(k), dim3(kWave), 0, st, n_waves, k, wcnt);
    if ((e = hipGetLastError()) != hipSuccess) return cleanup(e, "sl_eval_fmm: clustering launch");

    // ---- host: cubes, near/far lists, padded layout ---------------------------------------
    std::vector<unsigned long long> h_ext((size_t)6 * k), h_dmax(k);
    std::vector<unsigned int> h_cnt(k);
    double h_box[6];
    KmState h_st;
    e = hipMemcpyAsync(h_ext.data(), ext, h_ext.size() * 8, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipMemcpyAsync(h_dmax.data(), dmax, h_dmax.size() * 8, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipMemcpyAsync(h_cnt.data(), cnt, h_cnt.size() * 4, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipMemcpyAsync(h_box, gbox, sizeof(h_box), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipMemcpyAsync(&h_st, kst, sizeof(h_st), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return cleanup(e, "sl_eval_fmm: reading the clusters back");
    double gext = 0.0;
    for (int c = 0; c < 3; ++c) gext = std::max(gext, h_box[3 + c] - h_box[c]);
    const double amin = ldexp(gext, -20);
    std::vector<double> boxc((size_t)4 * k, 0.0), bdelta(k, 0.0);   // centre x, y, z, half width
    std::vector<int64_t> offs(k + 1, 0), cnts(k, 0);
    for (int j = 0; j < k; ++j) {
        cnts[j] = h_cnt[j];
        offs[j + 1] = offs[j] + round_up(cnts[j], kBoxPad);
        if (!cnts[j]) continue;
        double half = 0.0;
        for (int c = 0; c < 3; ++c) {
            const double lo = dec(h_ext[6 * j + c]), hi = dec(h_ext[6 * j + 3 + c]);
            const double sum = lo + hi;
            boxc[4 * j + c] = 0.5 * sum;
            const double span = hi - lo;
            half = std::max(half, span);
        }
        half = 0.5 * half;
        boxc[4 * j + 3] = std::max(half, amin);
        bdelta[j] = vard ? dec(h_dmax[j]) : delta;
    }
    const int64_t np = offs[k];
    // near[T][S]; an empty cluster has no points and no equivalent sources: near for every T, so
    // that the far-field pass never visits its (zero) equivalent records
    std::vector<uint8_t> nearm((size_t)k * k, 1);
    for (int T = 0; T < k; ++T) {
        if (!cnts[T]) continue;
        for (int S = 0; S < k; ++S) {
            if (!cnts[S]) continue;
            bool meets = true;
            double g[3];
            for (int c = 0; c < 3; ++c) {
                const double d = fabs(boxc[4 * T + c] - boxc[4 * S + c]);
                const double reach = kAlphaFar * boxc[4 * S + 3];
                const double lim = boxc[4 * T + 3] + reach;
                meets = meets && d <= lim;
                const double both = boxc[4 * T + 3] + boxc[4 * S + 3];
                const double gc = d - both;
                g[c] = gc > 0.0 ? gc : 0.0;
            }
            const double g0 = g[0] * g[0], g1 = g[1] * g[1], g2 = g[2] * g[2];
            const double g01 = g0 + g1;
            const double gap = sqrt(g01 + g2);
            const double cut = kRhoExact64 * bdelta[T];
            nearm[(size_t)T * k + S] = (T == S || meets || gap < cut) ? 1 : 0;
        }
    }
    // check points and equivalent points of every box (padded per box)
    const int pc = (int)round_up(ne, kBoxPad);     // check targets of a box: whole target groups
    const int pe = (int)round_up(ne, kCluster);    // equivalent sources of a box: whole clusters
    std::vector<double> chk((size_t)3 * k * pc), eqp((size_t)3 * k * pe);
    std::vector<int32_t> cperm((size_t)k * pc, -1), box_src_e((size_t)k * pe / kCluster),
        box_tgt_c((size_t)k * pc / kWave), box_surf((size_t)np / kWave);
    for (int j = 0; j < k; ++j) {
        const double *o = &boxc[4 * j];
        const double ac = kAlphaCheck * o[3], ae = kAlphaEq * o[3];
        for (int i = 0; i < pc; ++i)   // padding: copies of the box's first check point
            for (int c = 0; c < 3; ++c) {
                const double t = ac * E[3 * (i < ne ? i : 0) + c];
                chk[((size_t)j * pc + i) * 3 + c] = o[c] + t;
            }
        for (int i = 0; i < pe; ++i)
            for (int c = 0; c < 3; ++c) {
                const double t = i < ne ? ae * E[3 * i + c] : 0.0;
                eqp[((size_t)j * pe + i) * 3 + c] = o[c] + t;
            }
        for (int i = 0; i < ne; ++i) cperm[(size_t)j * pc + i] = j * ne + i;
        for (int c = 0; c < pe / kCluster; ++c) box_src_e[(size_t)j * (pe / kCluster) + c] = j;
        for (int c = 0; c < pc / kWave; ++c) box_tgt_c[(size_t)j * (pc / kWave) + c] = j;
        for (int64_t b = offs[j] / kWave; b < offs[j + 1] / kWave; ++b) box_surf[b] = j;
    }

    // ---- stage 2 workspace ------------------------------------------------------------------
    int R, wps;
    {
        std::lock_guard<std::mutex> l(ctx->mu);
        R = ctx->targets_per_lane;
        wps = ctx->waves_per_simd;
    }
    if (R == 0) R = mixed ? 1 : (np <= ((int64_t)1 << 17) ? 1 : 2);
    R = R > 2 ? 2 : R;   // the pair kernel's cluster-list instances keep at most two targets a lane
    // The cluster lists are shorter than the plain sum's source set: at most 64 waves per SIMD of
    // work items (measured at 92,256 points, FP64: 7.8 ms with 32 or 64, 8.6 ms with 128).
    const int waves_wanted = ctx->n_cu * 4 * std::min(wps, 64);
    PairPlan pn = plan_pairs(np, np, R, waves_wanted, mixed);                     // near field
    PairPlan pf = plan_pairs((int64_t)k * pe, np, R, waves_wanted, mixed);       // far field
    PairPlan pk = plan_pairs(np, (int64_t)k * pc, 1, waves_wanted, false);      // check potentials
    {
        // a box's check points take only that box's source clusters: no more ways than those
        int64_t most = 1;
        for (int j = 0; j < k; ++j) most = std::max(most, (offs[j + 1] - offs[j]) / kCluster);
        pk.n_ways = (int)std::min<int64_t>(pk.n_ways, most);
    }
    pn.n_cu = pf.n_cu = pk.n_cu = ctx->n_cu;
    const int64_t npc = (int64_t)k * pc, npe = (int64_t)k * pe;
    off = 0;
    const size_t b_x = take(np * 8), b_y = take(np * 8), b_z = take(np * 8);
    const size_t b_x32 = mixed ? take(np * 4) : 0, b_y32 = mixed ? take(np * 4) : 0, b_z32 = mixed ? take(np * 4) : 0;
    const size_t b_d = take(np * 64), b_f32 = mixed ? take(np * 32) : 0, b_dl = vard ? take(np * 8) : 0;
    const size_t b_perm = take(np * 4), b_sph = take(np / kCluster * sizeof(double4));
    const size_t b_off = take((size_t)(k + 1) * 8), b_cnts = take((size_t)k * 8), b_boxc = take((size_t)4 * k * 8);
    const size_t b_bdl = take((size_t)k * 8), b_near = take((size_t)k * k), b_bsurf = take((size_t)np / kWave * 4);
    const size_t b_cx = take(npc * 8), b_cy = take(npc * 8), b_cz = take(npc * 8), b_cperm = take(npc * 4);
    const size_t b_btc = take((size_t)npc / kWave * 4);
    const size_t b_vx = take((size_t)k * ne * 8), b_vy = take((size_t)k * ne * 8), b_vz = take((size_t)k * ne * 8);
    const size_t b_eqp = take((size_t)3 * npe * 8), b_erec = take(npe * 64), b_e32 = mixed ? take(npe * 32) : 0;
    const size_t b_esph = take(npe / kCluster * sizeof(double4)), b_bse = take((size_t)npe / kCluster * 4);
    const size_t b_centre = take(3 * 8);
    const size_t b_part = take((size_t)(pn.n_ways + pf.n_ways) * 3 * np * 8);
    const size_t b_cpart = take((size_t)pk.n_ways * 3 * npc * 8);
    const size_t b_tbs = take(tblock_scratch_bytes((int)(std::max(np, npc) / kWave)));
    e = ws_alloc(ctx, (void **)&B, off, st);
    if (e != hipSuccess) return cleanup(e, "sl_eval_fmm: workspace");
    auto at = [&](size_t o) { return B + o; };
    SortedOut so;
    so.x = (double *)at(b_x); so.y = (double *)at(b_y); so.z = (double *)at(b_z);
    so.x32 = mixed ? (float *)at(b_x32) : nullptr;
    so.y32 = mixed ? (float *)at(b_y32) : nullptr;
    so.z32 = mixed ? (float *)at(b_z32) : nullptr;
    so.d = (double *)at(b_d);
    so.f32 = mixed ? (float *)at(b_f32) : nullptr;
    so.delta = vard ? (double *)at(b_dl) : nullptr;
    so.perm = (int32_t *)at(b_perm);
    double4 *sph = (double4 *)at(b_sph);
    int64_t *d_off = (int64_t *)at(b_off), *d_cnts = (int64_t *)at(b_cnts);
    double *d_boxc = (double *)at(b_boxc), *d_bdl = (double *)at(b_bdl);
    uint8_t *d_near = (uint8_t *)at(b_near);
    int32_t *d_bsurf = (int32_t *)at(b_bsurf), *d_cperm = (int32_t *)at(b_cperm), *d_btc = (int32_t *)at(b_btc);
    double *d_eqp = (double *)at(b_eqp);
    double *cx = (double *)at(b_cx), *cy = (double *)at(b_cy), *cz = (double *)at(b_cz);
    double *vx = (double *)at(b_vx), *vy = (double *)at(b_vy), *vz = (double *)at(b_vz);
    double *erec = (double *)at(b_erec);
    float *e32 = mixed ? (float *)at(b_e32) : nullptr;
    double4 *esph = (double4 *)at(b_esph);
    int32_t *d_bse = (int32_t *)at(b_bse);
    double *part = (double *)at(b_part), *cpart = (double *)at(b_cpart);
    void *tbs = at(b_tbs);
    // uploads (pageable host memory: the copies complete before the calls return)
    struct Up { void *dst; const void *src; size_t bytes; };
    std::vector<double> gcentre = {0.5 * (h_box[0] + h_box[3]), 0.5 * (h_box[1] + h_box[4]), 0.5 * (h_box[2] + h_box[5])};
    std::vector<double> cxs(npc), cys(npc), czs(npc);
    for (int64_t i = 0; i < npc; ++i) { cxs[i] = chk[3 * i]; cys[i] = chk[3 * i + 1]; czs[i] = chk[3 * i + 2]; }
    double *d_centre = (double *)at(b_centre);
    const Up ups[] = {{d_off, offs.data(), offs.size() * 8}, {d_cnts, cnts.data(), cnts.size() * 8},
                      {d_boxc, boxc.data(), boxc.size() * 8}, {d_bdl, bdelta.data(), bdelta.size() * 8},
                      {d_near, nearm.data(), nearm.size()}, {d_bsurf, box_surf.data(), box_surf.size() * 4},
                      {cx, cxs.data(), cxs.size() * 8}, {cy, cys.data(), cys.size() * 8},
                      {cz, czs.data(), czs.size() * 8}, {d_cperm, cperm.data(), cperm.size() * 4},
                      {d_btc, box_tgt_c.data(), box_tgt_c.size() * 4}, {d_eqp, eqp.data(), eqp.size() * 8},
                      {d_bse, box_src_e.data(), box_src_e.size() * 4},
                      {d_centre, gcentre.data(), gcentre.size() * 8}};
    for (const Up &u : ups)
        if ((e = hipMemcpyAsync(u.dst, u.src, u.bytes, hipMemcpyHostToDevice, st)) != hipSuccess)
            return cleanup(e, "sl_eval_fmm: upload");
    // the host vectors above must outlive the copies
    if ((e = hipStreamSynchronize(st)) != hipSuccess) return cleanup(e, "sl_eval_fmm: upload");

    // ---- points in box order, records, spheres ---------------------------------------------
    hipLaunchKernelGGL(k_scatter_boxes, dim3(blocks_of(n, 256)), dim3(256), 0, st, x, y, z, w, fx, fy, fz, delta_tgt,
                       n, k, labels, rank, wcnt, d_off, d_centre, so);
    hipLaunchKernelGGL(k_pad_boxes, dim3(k), dim3(kBoxPad), 0, st, k, d_off, d_cnts, d_boxc, d_bdl, d_centre, so);
    hipLaunchKernelGGL(k_cluster_spheres, dim3((unsigned)(np / kCluster)), dim3(kWave), 0, st, so.d, sph);
    hipLaunchKernelGGL(k_equiv_records, dim3(blocks_of(npe, 256)), dim3(256), 0, st, npe, d_eqp, d_centre, erec, e32);
    if (labels_out)
        hipLaunchKernelGGL(k_copy_labels, dim3(blocks_of(n, 256)), dim3(256), 0, st, labels, n, labels_out);
    if ((e = hipGetLastError()) != hipSuccess) return cleanup(e, "sl_eval_fmm: packing launch");

    // ---- check potentials: each box's check points against its own points (plain Stokeslet) --
    PairArgs pa;
    pa.s = SrcView{so.d, nullptr, sph, np};
    TgtView tv{cx, cy, cz, nullptr, nullptr, nullptr, nullptr, d_cperm, npc, (int64_t)k * ne};
    pa.t = tv;
    pa.delta = 1.0;
    pa.far_cut = kRhoExact64;
    pa.rho64 = 0.0;
    pa.n_tblocks = pk.n_tblocks;
    pa.n_ways = pk.n_ways;
    pa.part = cpart;
    pa.bbox = gbox;
    pa.tblock_scratch = tbs;
    pa.records_ready = 0;
    pa.fmm_mode = 3;
    pa.fmm_k = k;
    pa.fmm_box_src = d_bsurf;
    pa.fmm_box_tgt = d_btc;
    pa.fmm_near = d_near;
    if ((e = launch_pair(pa, pk, false, false, st, nullptr)) != hipSuccess) return cleanup(e, "sl_eval_fmm: check potentials");
    if ((e = launch_reduce(cpart, pk.n_ways, npc, d_cperm, 1.0, vx, vy, vz, st)) != hipSuccess)
        return cleanup(e, "sl_eval_fmm: check potentials");
    hipLaunchKernelGGL(k_equiv_density, dim3(blocks_of((int64_t)k * 3 * ne, 256)), dim3(256), 0, st, k, ne, ne, Mdev,
                       vx, vy, vz, d_boxc, pe, erec, e32);
    hipLaunchKernelGGL(k_cluster_spheres, dim3((unsigned)(npe / kCluster)), dim3(kWave), 0, st, erec, esph);
    if ((e = hipGetLastError()) != hipSuccess) return cleanup(e, "sl_eval_fmm: equivalent densities");

    // ---- near field (regularized, near boxes) and far field (equivalent sources, far boxes) --
    TgtView ts{so.x, so.y, so.z, so.x32, so.y32, so.z32, so.delta, so.perm, np, n};
    double rho64;
    {
        std::lock_guard<std::mutex> l(ctx->mu);
        rho64 = ctx->rho64;
    }
    pa.s = SrcView{so.d, so.f32, sph, np};
    pa.t = ts;
    pa.delta = vard ? 1.0 : delta;
    pa.far_cut = mixed ? std::max(kRhoExact32, rho64) : kRhoExact64;
    pa.rho64 = rho64;
    pa.n_tblocks = pn.n_tblocks;
    pa.n_ways = pn.n_ways;
    pa.part = part;
    pa.fmm_mode = 1;
    pa.fmm_box_tgt = d_bsurf;
    if ((e = launch_pair(pa, pn, mixed, vard, st, nullptr)) != hipSuccess) return cleanup(e, "sl_eval_fmm: near field");
    pa.s = SrcView{erec, e32, esph, npe};
    pa.n_tblocks = pf.n_tblocks;
    pa.n_ways = pf.n_ways;
    pa.part = part + (size_t)pn.n_ways * 3 * np;
    pa.fmm_mode = 2;
    pa.fmm_box_src = d_bse;
    if ((e = launch_pair(pa, pf, mixed, vard, st, nullptr)) != hipSuccess) return cleanup(e, "sl_eval_fmm: far field");
    if ((e = launch_reduce(part, pn.n_ways + pf.n_ways, np, so.perm, 1.0 / (8.0 * M_PI * mu), ux, uy, uz, st)) !=
        hipSuccess)
        return cleanup(e, "sl_eval_fmm: reduction");
    const hipError_t e1 = hipFreeAsync(B, st), e2 = hipFreeAsync(A, st);
    if (e1 != hipSuccess) return hip_fail(e1, "sl_eval_fmm: hipFreeAsync");
    if (e2 != hipSuccess) return hip_fail(e2, "sl_eval_fmm: hipFreeAsync");
    return SL_OK;
}

}  // extern "C"
