// sl_internal.h -- host-side declarations shared by the library's translation units.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <atomic>
#include <condition_variable>
#include <deque>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "stokeslet.h"
#include "sl_device.h"

namespace sl {

// ---------------------------------------------------------------------------------------
// Error reporting
// ---------------------------------------------------------------------------------------
sl_status fail(sl_status s, const std::string &msg);
sl_status hip_fail(hipError_t e, const char *what);
#define SL_HIP(call)                                              \
    do {                                                          \
        hipError_t e_ = (call);                                   \
        if (e_ != hipSuccess) return ::sl::hip_fail(e_, #call);   \
    } while (0)

inline int64_t round_up(int64_t n, int64_t m) { return (n + m - 1) / m * m; }

// ---------------------------------------------------------------------------------------
// Sorted, padded point sets ("packed" layout in HBM)
// ---------------------------------------------------------------------------------------
// Sources after the spatial sort: np = round_up(n, kPad) entries; entries n..np-1 repeat the
// last real node with zero density.  Each source is one record of 8 words, x, y, z, gx, gy, gz,
// 0, 0 (g = w f), so that the pair kernel reads a source with one wide scalar load at a
// constant offset.  Clusters of 64 consecutive sources carry a bounding sphere (centre x, y, z,
// radius).
struct SrcView {
    const double *d;               // [np][8] double precision
    const float *f32;              // [np][8] single precision, positions minus the box centre
                                   // (mixed only)
    const double4 *sphere;         // [np / 64]
    int64_t np;
};

// Targets after the spatial sort, padded the same way.  perm[p] is the caller's index of
// sorted target p, or -1 for padding.
struct TgtView {
    const double *x, *y, *z;
    const float *x32, *y32, *z32;
    const double *delta;           // per-target delta (nullptr: scalar delta)
    const int32_t *perm;
    int64_t np;
    int64_t n;
};

struct PairArgs {
    SrcView s;
    TgtView t;
    double delta;            // scalar delta when t.delta == nullptr
    double far_cut;          // cluster far test: gap >= far_cut * delta_max
    double rho64;            // mixed path: pairs with r/delta below this are summed in FP64
    int n_tblocks;
    int n_ways;              // K: the clusters of a target block are dealt out to K waves by rank
    double *part;            // [n_ways][3][t.np] partial sums (unscaled)
    const double *bbox;      // [6] box of all points (min xyz, max xyz): bounds the rounding
                             // of the single-precision positions in the mixed path
    void *tblock_scratch;    // tblock_scratch_bytes(n_tblocks): per-target-block spheres
    int records_ready;       // 1: the source gather already wrote the target records (and
                             // zeroed the work counter), so launch_pair skips k_tblock
    // Single-level FMM (sl_fmm.hip): points grouped by cluster box, each box padded to whole
    // target groups and source clusters.  fmm_mode 0: every source cluster (the plain sum);
    // 1: only clusters of boxes near the target group's box; 2: only clusters of far boxes,
    // every pair plain (the far field from equivalent sources); 3: only clusters of the target
    // group's own box, every pair plain (check potentials).
    int fmm_mode = 0;
    int fmm_k = 0;                       // number of boxes
    const int32_t *fmm_box_src = nullptr;   // box of each source cluster of 64
    const int32_t *fmm_box_tgt = nullptr;   // box of each block of 64 targets
    const uint8_t *fmm_near = nullptr;      // [k][k]: box T near box S
};

// Optional events recorded around the pair kernel.
struct PairTiming {
    hipEvent_t e0, e1;
};
size_t tblock_scratch_bytes(int n_tblocks);

// Launch configuration chosen by the host for a given problem.
struct PairPlan {
    int R;                   // targets per lane
    int n_tblocks;
    int n_ways;
    int n_cu;                // compute units: the work loop launches an occupancy-sized grid
};

PairPlan plan_pairs(int64_t np_src, int64_t np_tgt, int R, int waves_wanted, bool mixed);
// Target blocks per workgroup of the pair kernel (they share one cluster stream).
int pair_group_size(bool mixed);
// The pair kernel's work counter inside tblock_scratch.
uint32_t *pair_counter(void *tblock_scratch, int n_tblocks);

hipError_t launch_pair(const PairArgs &a, const PairPlan &p, bool mixed, bool var_delta,
                       hipStream_t st, const PairTiming *tm);
hipError_t launch_reduce(const double *part, int n_ways, int64_t np, const int32_t *perm,
                         double scale, double *ux, double *uy, double *uz, hipStream_t st);
hipError_t launch_fill_zero(double *ux, double *uy, double *uz, int64_t n, hipStream_t st);

// sl_eval's validation and launch sequence (sl_api.hip).  fixed == nullptr: the workspace is
// allocated and freed stream-ordered; otherwise the fixed_bytes of device memory at `fixed` hold it
// (the number of ways is reduced until it fits; SL_EINVAL if even one way does not).  `who` names
// the entry point in error messages.
sl_status eval_common(const char *who, sl_ctx *ctx, sl_precision prec, int64_t n_src, const double *sx,
                      const double *sy, const double *sz, const double *w, const double *fx,
                      const double *fy, const double *fz, int64_t n_tgt, const double *tx,
                      const double *ty, const double *tz, double delta, const double *delta_tgt,
                      double mu, double *ux, double *uy, double *uz, void *stream, char *fixed,
                      size_t fixed_bytes);

// Per-patch regularization parameter (sl_patch.hip): out[p] = C delta*_i for the n x n nodes
// of each of n_patches patches (patch-major, row-major), n >= 1.
hipError_t launch_patch_delta(int64_t n_patches, int64_t n, const double *x, const double *y,
                              const double *z, double C, double *out, hipStream_t st);

// ---------------------------------------------------------------------------------------
// Packing: bounding box, Morton keys, stable radix sort, gather (sl_pack.hip)
// ---------------------------------------------------------------------------------------
struct PackScratch {
    uint32_t *keys[2];
    uint32_t *vals[2];
    uint32_t *counts[3];     // [256 * n_chunks] digit counts of each sort pass
    int64_t n_counts;
    double *bbox_part;       // [kBboxBlocks * 6]
    int n_bbox_parts;        // partials written by the last launch_bbox
    double *bbox;            // [6]: min x, y, z, max x, y, z
    double *centre;          // [3]: bounding-box centre (origin of the single-precision copies)
};

size_t sort_scratch_bytes(int64_t n);
void carve_sort_scratch(void *base, int64_t n, PackScratch &ps);

// Bounding box of up to two point sets (b may be empty): per-block partials, folded into
// ps.bbox / ps.centre by the first launch_sort_points that follows (before any reader).
hipError_t launch_bbox(const double *ax, const double *ay, const double *az, int64_t na,
                       const double *bx, const double *by, const double *bz, int64_t nb,
                       PackScratch &ps, hipStream_t st);
// Morton order of n points: on return *order points to n indices (sorted by key, stable).
hipError_t launch_sort_points(const double *x, const double *y, const double *z, int64_t n,
                              const PackScratch &ps, const uint32_t **order, hipStream_t st);

struct SrcOut {
    double *d;                                      // [np][8] source records
    float *f32;                                     // [np][8] single-precision records or nullptr
    double *x, *y, *z;                              // optional structure-of-arrays positions
    float *x32, *y32, *z32;                         // (targets = sources), nullptr if unused
    double4 *sphere;
    int32_t *perm;                                  // optional: sorted -> caller index (-1 pad)
};
// Target-group and target-block records of the pair kernel, written by the source gather when the
// targets are the sources (rec == nullptr: not written).  Needs R * G <= 4, so that a workgroup
// of 256 gathered points holds whole groups.
struct TRecOut {
    TBlockRec *rec;          // [n_groups] group records, then [n_tblocks] block records if G > 1
    uint32_t *ctr;           // the pair kernel's work counter, zeroed here
    const double *bbox;      // box of all points
    double gap_far;          // far_cut * delta
    int R, G, n_tblocks, mixed;
};
// g = w * f gathered in `order`; w may be nullptr when `wf_premul` (f already holds w*f).
hipError_t launch_gather_src(const uint32_t *order, int64_t n, int64_t np, const double *x,
                             const double *y, const double *z, const double *w, const double *fx,
                             const double *fy, const double *fz, const double *centre,
                             const SrcOut &o, const TRecOut &t, hipStream_t st);

struct TgtOut {
    double *x, *y, *z;
    float *x32, *y32, *z32;
    double *delta;
    int32_t *perm;
};
hipError_t launch_gather_tgt(const uint32_t *order, int64_t n, int64_t np, const double *x,
                             const double *y, const double *z, const double *delta_in,
                             const double *centre, const TgtOut &o, hipStream_t st);

// Gather only the density of a resident surface in its stored order (serving path).
hipError_t launch_gather_density(const int32_t *perm, int64_t n, int64_t np, const double *w,
                                 const double *fx, const double *fy, const double *fz,
                                 double *gx, double *gy, double *gz, float *gx32, float *gy32,
                                 float *gz32, hipStream_t st);

}  // namespace sl

// ---------------------------------------------------------------------------------------
// Context
// ---------------------------------------------------------------------------------------
struct sl_ctx;
namespace sl {
struct Server;   // serving runtime (sl_serve.hip)
// Fills the serving fields of `out` (zeros when the context never served).
void server_stats(sl_ctx *ctx, sl_stats *out);
}

struct sl_ctx {
    int device = 0;
    int n_cu = 0;
    size_t budget = 0;
    double rho64 = 0.0;
    int targets_per_lane = 0;   // 0: chosen per call
    int waves_per_simd = 128;
    std::mutex mu;
    sl::Server *server = nullptr;
    // pair-kernel timing (SL_PARAM_KERNEL_TIMING)
    bool timing = false;
    std::vector<sl::PairTiming> timed;   // recorded, not yet read
    std::vector<hipEvent_t> spare_events;
    uint64_t pair_launches = 0;
    double pair_ms = 0.0;
    // spline matrices of the upsampling step, per (n, factor): device memory, freed by sl_destroy
    std::unordered_map<int64_t, double *> splines;
    // unit-box operators of the single-level FMM, per points per cube edge: device memory
    std::unordered_map<int, double *> fmm_ops;
    // Stream-ordered workspaces come from this pool, which keeps what it has allocated until the
    // context is destroyed: the device's default pool returns its memory at every synchronization,
    // and a caller that synchronizes between calls would pay a fresh allocation each time.
    hipMemPool_t pool = nullptr;
};

namespace sl {
// Workspace of `bytes` from the context's pool, stream-ordered on `st` (freed with hipFreeAsync).
inline hipError_t ws_alloc(sl_ctx *ctx, void **p, size_t bytes, hipStream_t st)
{
    return hipMallocFromPoolAsync(p, bytes, ctx->pool, st);
}
}
