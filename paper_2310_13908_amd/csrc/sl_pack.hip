// sl_pack.hip -- staging of the inputs of the single-layer sum on gfx950.
//
// The pair kernels classify whole blocks of targets against clusters of 64 sources as
// "far" (plain Stokeslet, no erf/exp) or "near" (regularized), which only pays off when
// consecutive points are close in space.  Packing therefore:
//   1. takes the bounding box of all points (partials per block, folded in a fixed order by the
//      Morton-key kernel: deterministic),
//   2. orders the points along a 24-bit Morton curve (stable LSD radix sort, three passes of
//      8-bit digits; each pass's digit histogram is counted by the kernel that writes the
//      pass's input, so a pass is two launches: scan and scatter).  Up to 2^16 points the
//      lowest digit is skipped: 2^16 cells of the curve's top 16 bits are already finer than
//      the points, and points that share a cell keep their input order,
//   3. gathers positions and the packed density g = w f (the trapezoid-POU weight of
//      Sec. 3.3 folded into the force) into padded per-source records, plus the
//      single-precision records used by the mixed path (positions relative to the box centre),
//   4. computes one bounding sphere per cluster of 64 sources.
// Everything is O(N) and runs on the caller's stream.
#include "sl_internal.h"

namespace sl {

namespace {

constexpr int kBboxBlocks = 256;
constexpr int kBboxThreads = 256;
constexpr int kSortThreads = 256;
constexpr int kSortItems = 4;
constexpr int kSortChunk = kSortThreads * kSortItems;   // elements per block and pass
constexpr int kMortonBits = 8;                          // per axis
constexpr int kDigitBits = 8;
constexpr int kPasses = 3 * kMortonBits / kDigitBits;
constexpr int64_t kTwoPassMaxN = 1 << 16;   // up to this many points, sort by the top 16 bits
constexpr int kSortBlocksNoScan = 64;   // up to this many blocks, the scatters scan for themselves

// ----------------------------------------------------------------------------------------
// Bounding box
// ----------------------------------------------------------------------------------------
__global__ __launch_bounds__(kBboxThreads) void k_bbox_partial(
    const double *__restrict__ ax, const double *__restrict__ ay, const double *__restrict__ az,
    int64_t na, const double *__restrict__ bx, const double *__restrict__ by,
    const double *__restrict__ bz, int64_t nb, double *__restrict__ part,
    uint32_t *__restrict__ zero, int64_t n_zero)
{
    double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    // the first sort's digit counters, counted by k_morton after this kernel
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n_zero; i += stride) zero[i] = 0u;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < na + nb; i += stride) {
        double p[3];
        if (i < na) { p[0] = ax[i]; p[1] = ay[i]; p[2] = az[i]; }
        else { p[0] = bx[i - na]; p[1] = by[i - na]; p[2] = bz[i - na]; }
#pragma unroll
        for (int k = 0; k < 3; ++k) { lo[k] = fmin(lo[k], p[k]); hi[k] = fmax(hi[k], p[k]); }
    }
    __shared__ double red[6][kBboxThreads / kWave];
    const int w = threadIdx.x / kWave, lane = threadIdx.x % kWave;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const double l = wave_min(lo[k]), h = wave_max(hi[k]);
        if (lane == 0) { red[k][w] = l; red[3 + k][w] = h; }
    }
    __syncthreads();
    if (threadIdx.x < 6) {
        const int k = threadIdx.x;
        double v = red[k][0];
        for (int j = 1; j < kBboxThreads / kWave; ++j) v = k < 3 ? fmin(v, red[k][j]) : fmax(v, red[k][j]);
        part[blockIdx.x * 6 + k] = v;
    }
}

// ----------------------------------------------------------------------------------------
// Morton keys
// ----------------------------------------------------------------------------------------
__device__ __forceinline__ uint32_t quantize(double v, double lo, double hi)
{
    const double span = hi - lo;
    double t = span > 0.0 ? (v - lo) / span : 0.0;
    t = t * (double)(1 << kMortonBits);
    int q = (int)t;
    q = q < 0 ? 0 : (q > (1 << kMortonBits) - 1 ? (1 << kMortonBits) - 1 : q);
    return (uint32_t)q;
}

// Interleave: bit b of axis a goes to key bit 3 b + (2 - a)  (x is the most significant).
__device__ __forceinline__ uint32_t morton3(uint32_t qx, uint32_t qy, uint32_t qz)
{
    uint32_t k = 0;
#pragma unroll
    for (int b = 0; b < kMortonBits; ++b) {
        k |= ((qx >> b) & 1u) << (3 * b + 2);
        k |= ((qy >> b) & 1u) << (3 * b + 1);
        k |= ((qz >> b) & 1u) << (3 * b + 0);
    }
    return k;
}

// Clears the counts of sort passes 1 and 2.  Every block first folds the bounding-box partials (in the same order, so every block gets the
// same box; block 0 also stores it with its centre for the later kernels).  Then: keys, identity
// values, and the digit counts of the first sort pass (counts[digit * nblocks + block], block =
// i / kSortChunk; integer atomics, so the counts do not depend on their order).
__global__ __launch_bounds__(256) void k_morton(const double *__restrict__ x,
                                                const double *__restrict__ y,
                                                const double *__restrict__ z, int64_t n,
                                                const double *__restrict__ bbox_part, int nparts,
                                                double *__restrict__ bbox_out,
                                                double *__restrict__ centre_out,
                                                uint32_t *__restrict__ keys,
                                                uint32_t *__restrict__ vals,
                                                uint32_t *__restrict__ counts, int nblocks,
                                                int shift0, uint32_t *__restrict__ clear1,
                                                uint32_t *__restrict__ clear2, int64_t n_clear)
{
    __shared__ double box[6];
    // the counts of sort passes 1 and 2, accumulated by the scatters of passes 0 and 1
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n_clear;
         i += (int64_t)gridDim.x * blockDim.x) {
        clear1[i] = 0u;
        clear2[i] = 0u;
    }
    __shared__ double red[4][6];
    {   // one partial per thread (nparts <= 256), min / max over the block: order-independent
        double v[6];
        for (int k = 0; k < 6; ++k) v[k] = k < 3 ? INFINITY : -INFINITY;
        if ((int)threadIdx.x < nparts)
            for (int k = 0; k < 6; ++k) v[k] = bbox_part[threadIdx.x * 6 + k];
        for (int k = 0; k < 6; ++k) v[k] = k < 3 ? wave_min(v[k]) : wave_max(v[k]);
        const int wv = threadIdx.x / kWave;
        if (threadIdx.x % kWave == 0)
            for (int k = 0; k < 6; ++k) red[wv][k] = v[k];
        __syncthreads();
        if (threadIdx.x < 6) {
            const int k = threadIdx.x;
            double r = red[0][k];
            for (int j = 1; j < 4; ++j) r = k < 3 ? fmin(r, red[j][k]) : fmax(r, red[j][k]);
            box[k] = r;
        }
        __syncthreads();
    }
    if (blockIdx.x == 0 && threadIdx.x < 6) {
        bbox_out[threadIdx.x] = box[threadIdx.x];
        if (threadIdx.x < 3) centre_out[threadIdx.x] = 0.5 * (box[threadIdx.x] + box[threadIdx.x + 3]);
    }
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const uint32_t qx = quantize(x[i], box[0], box[3]);
        const uint32_t qy = quantize(y[i], box[1], box[4]);
        const uint32_t qz = quantize(z[i], box[2], box[5]);
        const uint32_t k = morton3(qx, qy, qz);
        keys[i] = k;
        vals[i] = (uint32_t)i;
        atomicAdd(&counts[(int64_t)((k >> shift0) & 255u) * nblocks + i / kSortChunk], 1u);
    }
}

// ----------------------------------------------------------------------------------------
// Stable LSD radix sort of (key, value) pairs, 8-bit digits.
// Block b owns elements [b * kSortChunk, (b + 1) * kSortChunk) in every pass.  The counts of
// pass p live in their own buffer, counted by the kernel that writes pass p's input.
// ----------------------------------------------------------------------------------------
// Exclusive scan of the (digit, block) counts of a pass for many blocks, in three launches:
// per-segment sums (k_scan_sums, which also clears the next pass's counts), their exclusive
// scan in one workgroup (k_scan_top), and the segment scans plus their offsets (k_scan_apply).
// Integer sums: the result does not depend on the order.
constexpr int kScanThreads = 1024;
constexpr int kScanSeg = 4 * kScanThreads;   // counters per segment (four per thread)

// Exclusive scan of one value per thread across the workgroup; returns the workgroup total.
__device__ uint32_t block_exclusive_scan(uint32_t v, uint32_t &excl, uint32_t *sh)
{
    const int t = threadIdx.x, lane = t % kWave, w = t / kWave;
    uint32_t incl = v;
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
        const uint32_t u = __shfl_up(incl, o, kWave);
        incl += lane >= o ? u : 0u;
    }
    if (lane == kWave - 1) sh[w] = incl;
    __syncthreads();
    uint32_t base = 0, total = 0;
    for (int j = 0; j < (int)(blockDim.x / kWave); ++j) {
        base += j < w ? sh[j] : 0u;
        total += sh[j];
    }
    __syncthreads();
    excl = base + incl - v;
    return total;
}

__global__ __launch_bounds__(kScanThreads) void k_scan_sums(const uint32_t *__restrict__ c, int64_t total,
                                                            uint32_t *__restrict__ part,
                                                            uint32_t *__restrict__ next)
{
    __shared__ uint32_t sh[kScanThreads / kWave];
    for (int64_t i = (int64_t)blockIdx.x * kScanThreads + threadIdx.x; i < total;
         i += (int64_t)gridDim.x * kScanThreads)
        next[i] = 0u;
    const int64_t base = (int64_t)blockIdx.x * kScanSeg;
    uint32_t v = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const int64_t i = base + k * kScanThreads + threadIdx.x;
        v += i < total ? c[i] : 0u;
    }
    uint32_t excl;
    const uint32_t tot = block_exclusive_scan(v, excl, sh);
    if (threadIdx.x == 0) part[blockIdx.x] = tot;
}

__global__ __launch_bounds__(kScanThreads) void k_scan_top(uint32_t *__restrict__ part, int n)
{
    __shared__ uint32_t sh[kScanThreads / kWave];
    const int per = (n + kScanThreads - 1) / kScanThreads;
    const int b = threadIdx.x * per, e = b + per < n ? b + per : n;
    uint32_t v = 0;
    for (int i = b; i < e; ++i) v += part[i];
    uint32_t run;
    block_exclusive_scan(v, run, sh);
    for (int i = b; i < e; ++i) {
        const uint32_t c = part[i];
        part[i] = run;
        run += c;
    }
}

__global__ __launch_bounds__(kScanThreads) void k_scan_apply(uint32_t *__restrict__ c, int64_t total,
                                                             const uint32_t *__restrict__ part)
{
    __shared__ uint32_t sh[kScanThreads / kWave];
    const int64_t i0 = (int64_t)blockIdx.x * kScanSeg + 4 * (int64_t)threadIdx.x;
    uint32_t x[4], v = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        x[k] = i0 + k < total ? c[i0 + k] : 0u;
        v += x[k];
    }
    uint32_t run;
    block_exclusive_scan(v, run, sh);
    run += part[blockIdx.x];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        if (i0 + k < total) c[i0 + k] = run;
        run += x[k];
    }
}

// Scatter by the digit at `shift`; when `next` is set, also counts the digit at shift + 8 of
// every element for the block that owns its new position.  `offs` holds the pass's counts,
// exclusively scanned by k_scan_* when `scanned`; otherwise (few blocks) every block takes its
// offsets from the raw counts itself: for digit d, the counts of all digits below d plus those
// of digit d in the blocks before it.
__global__ __launch_bounds__(kSortThreads) void k_rs_scatter(
    const uint32_t *__restrict__ kin, const uint32_t *__restrict__ vin,
    uint32_t *__restrict__ kout, uint32_t *__restrict__ vout, int64_t n, int shift,
    const uint32_t *__restrict__ offs, int scanned, int nblocks, uint32_t *__restrict__ next,
    uint32_t *__restrict__ clear)
{
    static_assert(kSortThreads == 256, "one thread per digit");
    constexpr int kWaves = kSortThreads / kWave;
    __shared__ uint32_t base[256];
    __shared__ uint32_t cnt[kWaves][256];
    const int t = threadIdx.x, w = t / kWave, lane = t % kWave;
    if (clear)   // the first pass's counts, for a following sort
        clear[(int64_t)t * nblocks + blockIdx.x] = 0u;
    if (scanned) {
        base[t] = offs[(int64_t)t * nblocks + blockIdx.x];
    } else {
        uint32_t row = 0, before = 0;
#pragma unroll 16
        for (int b = 0; b < nblocks; ++b) {
            const uint32_t c = offs[(int64_t)t * nblocks + b];
            row += c;
            before += b < (int)blockIdx.x ? c : 0u;
        }
        // exclusive scan of the digit totals: within each wave, then across the four waves
        uint32_t incl = row;
#pragma unroll
        for (int o = 1; o < kWave; o <<= 1) {
            const uint32_t v = __shfl_up(incl, o, kWave);
            incl += lane >= o ? v : 0u;
        }
        if (lane == kWave - 1) cnt[0][w] = incl;
        __syncthreads();
        uint32_t wbase = 0;
        for (int j = 0; j < w; ++j) wbase += cnt[0][j];
        base[t] = wbase + incl - row + before;
        __syncthreads();
    }
    const uint64_t lt = lane == 0 ? 0ull : (~0ull >> (64 - lane));
    const int64_t start = (int64_t)blockIdx.x * kSortChunk;
    for (int k = 0; k < kSortItems; ++k) {
        const int64_t i = start + k * kSortThreads + t;
        const bool valid = i < n;
        const uint32_t key = valid ? kin[i] : 0u;
        const uint32_t val = valid ? vin[i] : 0u;
        const uint32_t d = (key >> shift) & 255u;
        // Lanes of this wave holding the same digit.
        uint64_t peers = __ballot(valid);
#pragma unroll
        for (int bit = 0; bit < 8; ++bit) {
            const bool set = (d >> bit) & 1u;
            const uint64_t m = __ballot(set);
            peers &= set ? m : ~m;
        }
        const uint32_t rank = __popcll(peers & lt);
        const uint32_t wcount = __popcll(peers);
#pragma unroll
        for (int j = 0; j < kWaves; ++j) cnt[j][t] = 0;
        __syncthreads();
        if (valid && rank == 0) cnt[w][d] = wcount;
        __syncthreads();
        if (valid) {
            uint32_t off = base[d] + rank;
            for (int j = 0; j < w; ++j) off += cnt[j][d];
            kout[off] = key;
            vout[off] = val;
            if (next)
                atomicAdd(&next[(int64_t)((key >> (shift + kDigitBits)) & 255u) * nblocks + off / kSortChunk], 1u);
        }
        __syncthreads();
        uint32_t add = 0;
#pragma unroll
        for (int j = 0; j < kWaves; ++j) add += cnt[j][t];
        base[t] += add;
        __syncthreads();
    }
}

// ----------------------------------------------------------------------------------------
// Gathers
// ----------------------------------------------------------------------------------------
// One wave per cluster of 64 sorted sources: gather, pack g = w f, cluster bounding sphere.
__global__ __launch_bounds__(256) void k_gather_src(
    const uint32_t *__restrict__ order, int64_t n, int64_t np, const double *__restrict__ x,
    const double *__restrict__ y, const double *__restrict__ z, const double *__restrict__ w,
    const double *__restrict__ fx, const double *__restrict__ fy, const double *__restrict__ fz,
    const double *__restrict__ centre, SrcOut o, TRecOut t)
{
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;   // np % 256 == 0
    const bool real = p < n;
    const uint32_t idx = order[real ? p : n - 1];
    const double px = x[idx], py = y[idx], pz = z[idx];
    const double wt = real ? w[idx] : 0.0;
    const double gx = wt * fx[idx], gy = wt * fy[idx], gz = wt * fz[idx];
    double4 *rd = reinterpret_cast<double4 *>(o.d + p * 8);
    rd[0] = make_double4(px, py, pz, gx);
    rd[1] = make_double4(gy, gz, 0.0, 0.0);
    const float qx = (float)(px - centre[0]), qy = (float)(py - centre[1]), qz = (float)(pz - centre[2]);
    if (o.f32) {
        float4 *rf = reinterpret_cast<float4 *>(o.f32 + p * 8);
        rf[0] = make_float4(qx, qy, qz, (float)gx);
        rf[1] = make_float4((float)gy, (float)gz, 0.0f, 0.0f);
    }
    if (o.x) { o.x[p] = px; o.y[p] = py; o.z[p] = pz; }
    if (o.x32) { o.x32[p] = qx; o.y32[p] = qy; o.z32[p] = qz; }
    if (o.perm) o.perm[p] = real ? (int32_t)idx : -1;
    // Cluster sphere: centre of the cluster's box, radius = farthest member (+ a relative
    // margin so that rounding never shrinks it).
    const double lo[3] = {wave_min(px), wave_min(py), wave_min(pz)};
    const double hi[3] = {wave_max(px), wave_max(py), wave_max(pz)};
    const double cx = 0.5 * (lo[0] + hi[0]), cy = 0.5 * (lo[1] + hi[1]), cz = 0.5 * (lo[2] + hi[2]);
    const double dx = px - cx, dy = py - cy, dz = pz - cz;
    const double rad = sqrt(wave_max(dx * dx + dy * dy + dz * dz)) * (1.0 + 0x1p-40);
    const int lane = threadIdx.x % kWave, wv = threadIdx.x / kWave;
    if (lane == 0) o.sphere[p / kCluster] = make_double4(cx, cy, cz, rad);
    if (!t.rec) return;
    // Targets = sources: the pair kernel's target-group and target-block spheres from the same
    // points (box centre, farthest member, margin), as its own record kernel computes them.
    __shared__ double sh[4][8];
    if (lane == 0)
        for (int k = 0; k < 3; ++k) { sh[wv][k] = lo[k]; sh[wv][3 + k] = hi[k]; }
    __syncthreads();
    const int R = t.R, RG = t.R * t.G;
    const int wb = wv / R * R, wg = wv / RG * RG;    // first wave of this block / group
    double bl[3], bh[3], gl[3], gh[3];
    for (int k = 0; k < 3; ++k) { bl[k] = gl[k] = INFINITY; bh[k] = gh[k] = -INFINITY; }
    for (int v = wg; v < wg + RG; ++v)
        for (int k = 0; k < 3; ++k) {
            gl[k] = fmin(gl[k], sh[v][k]); gh[k] = fmax(gh[k], sh[v][3 + k]);
            if (v >= wb && v < wb + R) { bl[k] = fmin(bl[k], sh[v][k]); bh[k] = fmax(bh[k], sh[v][3 + k]); }
        }
    const double bx = 0.5 * (bl[0] + bh[0]), by = 0.5 * (bl[1] + bh[1]), bz = 0.5 * (bl[2] + bh[2]);
    const double gx0 = 0.5 * (gl[0] + gh[0]), gy0 = 0.5 * (gl[1] + gh[1]), gz0 = 0.5 * (gl[2] + gh[2]);
    const double ex = px - bx, ey = py - by, ez = pz - bz;
    const double fx0 = px - gx0, fy0 = py - gy0, fz0 = pz - gz0;
    const double rb = wave_max(fma(ex, ex, fma(ey, ey, __dmul_rn(ez, ez))));
    const double rg = wave_max(fma(fx0, fx0, fma(fy0, fy0, __dmul_rn(fz0, fz0))));
    __syncthreads();                 // every wave has read the boxes
    if (lane == 0) { sh[wv][6] = rb; sh[wv][7] = rg; }
    __syncthreads();
    double gap_far = t.gap_far;
    if (t.mixed) {
        const double ux = t.bbox[3] - t.bbox[0], uy = t.bbox[4] - t.bbox[1], uz = t.bbox[5] - t.bbox[2];
        gap_far = fmax(gap_far, 0x1p-10 * sqrt(fma(ux, ux, fma(uy, uy, __dmul_rn(uz, uz)))));
    }
    const int n_groups = t.n_tblocks / t.G;
    if (lane == 0 && wv == wg) {
        double r2 = 0.0;
        for (int v = wg; v < wg + RG; ++v) r2 = fmax(r2, sh[v][7]);
        TBlockRec rec = {gx0, gy0, gz0, sqrt(r2) * (1.0 + 0x1p-40), gap_far, gap_far, 0.0, 0.0};
        t.rec[blockIdx.x * (4 / RG) + wv / RG] = rec;
    }
    if (t.G > 1 && lane == 0 && wv == wb) {
        double r2 = 0.0;
        for (int v = wb; v < wb + R; ++v) r2 = fmax(r2, sh[v][6]);
        TBlockRec rec = {bx, by, bz, sqrt(r2) * (1.0 + 0x1p-40), gap_far, gap_far, 0.0, 0.0};
        t.rec[n_groups + blockIdx.x * (4 / R) + wv / R] = rec;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) *t.ctr = 0u;
}

__global__ __launch_bounds__(256) void k_gather_tgt(
    const uint32_t *__restrict__ order, int64_t n, const double *__restrict__ x,
    const double *__restrict__ y, const double *__restrict__ z,
    const double *__restrict__ delta_in, const double *__restrict__ centre, TgtOut o)
{
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const bool real = p < n;
    const uint32_t idx = order[real ? p : n - 1];
    if (o.x) {   // positions (absent when only the per-target delta is gathered)
        const double px = x[idx], py = y[idx], pz = z[idx];
        o.x[p] = px; o.y[p] = py; o.z[p] = pz;
        if (o.x32) {
            o.x32[p] = (float)(px - centre[0]);
            o.y32[p] = (float)(py - centre[1]);
            o.z32[p] = (float)(pz - centre[2]);
        }
    }
    if (o.delta) o.delta[p] = delta_in[idx];
    if (o.perm) o.perm[p] = real ? (int32_t)idx : -1;
}

__global__ __launch_bounds__(256) void k_gather_density(
    const int32_t *__restrict__ perm, int64_t np, const double *__restrict__ w_sorted,
    const double *__restrict__ fx, const double *__restrict__ fy, const double *__restrict__ fz,
    double *__restrict__ gx, double *__restrict__ gy, double *__restrict__ gz,
    float *__restrict__ gx32, float *__restrict__ gy32, float *__restrict__ gz32)
{
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= np) return;
    const int32_t idx = perm[p];
    double a = 0.0, b = 0.0, c = 0.0;
    if (idx >= 0) {
        const double wt = w_sorted[p];
        a = wt * fx[idx]; b = wt * fy[idx]; c = wt * fz[idx];
    }
    gx[p] = a; gy[p] = b; gz[p] = c;
    if (gx32) { gx32[p] = (float)a; gy32[p] = (float)b; gz32[p] = (float)c; }
}

int sort_blocks(int64_t n) { return (int)((n + kSortChunk - 1) / kSortChunk); }

}  // namespace

// ----------------------------------------------------------------------------------------
// Host wrappers
// ----------------------------------------------------------------------------------------
size_t sort_scratch_bytes(int64_t n)
{
    const int64_t nb = sort_blocks(n > 0 ? n : 1);
    size_t b = 0;
    b += 4 * round_up(n * 4, 256);                 // keys[2], vals[2]
    b += 3 * round_up(256 * nb * 4, 256);          // counts of the three passes
    b += round_up(kBboxBlocks * 6 * 8, 256);       // bbox partials
    b += 256 + 256;                                // bbox, centre
    return b;
}

void carve_sort_scratch(void *base, int64_t n, PackScratch &ps)
{
    char *p = static_cast<char *>(base);
    const int64_t nb = sort_blocks(n > 0 ? n : 1);
    for (int k = 0; k < 2; ++k) { ps.keys[k] = (uint32_t *)p; p += round_up(n * 4, 256); }
    for (int k = 0; k < 2; ++k) { ps.vals[k] = (uint32_t *)p; p += round_up(n * 4, 256); }
    for (int k = 0; k < 3; ++k) { ps.counts[k] = (uint32_t *)p; p += round_up(256 * nb * 4, 256); }
    ps.n_counts = 256 * nb;
    ps.bbox_part = (double *)p; p += round_up(kBboxBlocks * 6 * 8, 256);
    ps.bbox = (double *)p; p += 256;
    ps.centre = (double *)p;
}

hipError_t launch_bbox(const double *ax, const double *ay, const double *az, int64_t na,
                       const double *bx, const double *by, const double *bz, int64_t nb,
                       PackScratch &ps, hipStream_t st)
{
    const int64_t tot = na + nb;
    int blocks = (int)((tot + kBboxThreads - 1) / kBboxThreads);
    blocks = blocks < 1 ? 1 : (blocks > kBboxBlocks ? kBboxBlocks : blocks);
    hipLaunchKernelGGL(k_bbox_partial, dim3(blocks), dim3(kBboxThreads), 0, st, ax, ay, az, na,
                       bx, by, bz, nb, ps.bbox_part, ps.counts[0], ps.n_counts);
    ps.n_bbox_parts = blocks;   // folded by k_morton
    return hipGetLastError();
}

// k_morton counts the first pass's digits into counts[0] (cleared by k_bbox_partial) and clears
// counts[1] and counts[2]; the scatter of pass p counts into counts[p + 1], and the last one
// clears counts[0] for a following sort.  With more than kSortBlocksNoScan blocks, the three
// k_scan_* kernels scan counts[p] before pass p (and clear counts[(p + 1) % 3] as well).
hipError_t launch_sort_points(const double *x, const double *y, const double *z, int64_t n,
                              const PackScratch &ps, const uint32_t **order, hipStream_t st)
{
    const int nb = sort_blocks(n);
    const int64_t mb = (n + 255) / 256;
    const int passes = n <= kTwoPassMaxN ? kPasses - 1 : kPasses;
    const int shift0 = (kPasses - passes) * kDigitBits;
    hipLaunchKernelGGL(k_morton, dim3((unsigned)(mb < 1024 ? mb : 1024)), dim3(256), 0, st, x, y, z, n,
                       ps.bbox_part, ps.n_bbox_parts, ps.bbox, ps.centre, ps.keys[0], ps.vals[0],
                       ps.counts[0], nb, shift0, ps.counts[1], ps.counts[2], (int64_t)256 * nb);
    // With few blocks every scatter block sums the raw counts itself (at most 64 per thread), and
    // the single-workgroup scan launches are skipped.
    const bool scan = nb > kSortBlocksNoScan;
    int cur = 0;
    for (int p = 0; p < passes; ++p) {
        if (scan) {
            // counts[(p + 2) % 3] (the previous pass's, consumed; pass 2's before pass 0, which
            // k_scan_sums of pass 1 clears again) holds the segment sums
            const int64_t total = (int64_t)256 * nb;
            const int nseg = (int)((total + kScanSeg - 1) / kScanSeg);
            uint32_t *part = ps.counts[(p + 2) % 3];
            hipLaunchKernelGGL(k_scan_sums, dim3(nseg), dim3(kScanThreads), 0, st, ps.counts[p], total, part,
                               ps.counts[(p + 1) % 3]);
            hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(kScanThreads), 0, st, part, nseg);
            hipLaunchKernelGGL(k_scan_apply, dim3(nseg), dim3(kScanThreads), 0, st, ps.counts[p], total, part);
        }
        hipLaunchKernelGGL(k_rs_scatter, dim3(nb), dim3(kSortThreads), 0, st, ps.keys[cur],
                           ps.vals[cur], ps.keys[cur ^ 1], ps.vals[cur ^ 1], n, shift0 + p * kDigitBits,
                           ps.counts[p], scan ? 1 : 0, nb, p + 1 < passes ? ps.counts[p + 1] : nullptr,
                           p + 1 == passes ? ps.counts[0] : nullptr);
        cur ^= 1;
    }
    *order = ps.vals[cur];
    return hipGetLastError();
}

hipError_t launch_gather_src(const uint32_t *order, int64_t n, int64_t np, const double *x,
                             const double *y, const double *z, const double *w, const double *fx,
                             const double *fy, const double *fz, const double *centre,
                             const SrcOut &o, const TRecOut &t, hipStream_t st)
{
    if (t.rec && (t.R * t.G > 4 || 4 % (t.R * t.G) != 0)) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_gather_src, dim3((unsigned)(np / 256)), dim3(256), 0, st, order, n, np,
                       x, y, z, w, fx, fy, fz, centre, o, t);
    return hipGetLastError();
}

hipError_t launch_gather_tgt(const uint32_t *order, int64_t n, int64_t np, const double *x,
                             const double *y, const double *z, const double *delta_in,
                             const double *centre, const TgtOut &o, hipStream_t st)
{
    hipLaunchKernelGGL(k_gather_tgt, dim3((unsigned)(np / 256)), dim3(256), 0, st, order, n, x, y,
                       z, delta_in, centre, o);
    return hipGetLastError();
}

hipError_t launch_gather_density(const int32_t *perm, int64_t n, int64_t np, const double *w,
                                 const double *fx, const double *fy, const double *fz,
                                 double *gx, double *gy, double *gz, float *gx32, float *gy32,
                                 float *gz32, hipStream_t st)
{
    (void)n;
    hipLaunchKernelGGL(k_gather_density, dim3((unsigned)((np + 255) / 256)), dim3(256), 0, st,
                       perm, np, w, fx, fy, fz, gx, gy, gz, gx32, gy32, gz32);
    return hipGetLastError();
}

}  // namespace sl
