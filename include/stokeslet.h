/*
 * stokeslet.h -- C ABI of the MI355X (gfx950) regularized Stokes single-layer library.
 *
 * The operation (Agarwal & Biros, Sec. 3.4, eq. (regstokes), discretized with the
 * trapezoid-POU rule of Sec. 3.3, eq. (smoothint)):
 *
 *   u_i = 1/(8 pi mu) * sum_j w_j [ s1(r/d)/r f_j + s2(r/d)/r^3 (f_j . x_ij) x_ij ],
 *   x_ij = t_i - x_j,  r = |x_ij|,  d = delta (or delta_tgt[i]),
 *   s1(p) = erf p - (2/3) p (2p^2 - 5) e^{-p^2}/sqrt(pi),
 *   s2(p) = erf p - (2/3) p (4p^4 - 14p^2 + 3) e^{-p^2}/sqrt(pi),
 *
 * with the r = 0 limit s1(r/d)/r -> 16/(3 d sqrt(pi)) (Sec. 3.4); the pair with r = 0
 * contributes only that term.  Every source is summed for every target, including a
 * target that coincides with a source.
 *
 * Conventions shared by every entry point:
 *  - Arrays are structure-of-arrays, IEEE double, in DEVICE memory of the context's GPU
 *    (e.g. torch tensors' data_ptr()).  Positions and densities are not scanned: NaN/Inf
 *    propagate into the affected outputs.
 *  - The caller owns every array it passes; the library never frees caller memory.
 *    Arrays passed to an asynchronous call must stay valid until that work completes.
 *  - Outputs must not alias inputs.
 *  - A status code is returned; on failure sl_last_error() gives a message (per thread).
 *    Invalid arguments are rejected before any GPU work is enqueued.
 */
#ifndef STOKESLET_H
#define STOKESLET_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    SL_OK = 0,
    SL_EINVAL = -1,     /* bad argument: NULL pointer, n < 0, delta/mu not finite and > 0, aliasing */
    SL_ENOMEM = -2,     /* device allocation failed */
    SL_EBUSY = -3,      /* admission refused: the HBM budget is exhausted */
    SL_EHIP = -4,       /* a HIP runtime call or a kernel launch failed */
    SL_ENOTFOUND = -5,  /* unknown surface handle or request id */
    SL_ETIMEDOUT = -6   /* sl_wait gave up before the request completed */
} sl_status;

typedef enum {
    SL_FP64 = 0,        /* every pair in double precision; ~1e-15 relative to the exact sum */
    SL_MIXED = 1        /* pairs with rho = r/delta >= rho64 in single precision (smoothed for
                           rho < 5 from a table of cubics in rho^2, plain Stokeslet beyond, where
                           s1 = s2 = 1 to single precision), summed per cluster of 64 sources and
                           folded into a per-target two-sum (hi, lo) pair; pairs with rho < rho64
                           (default 0: none) and the final per-target sum in double precision;
                           ~1e-7 relative */
} sl_precision;

typedef struct sl_ctx sl_ctx;   /* opaque; one per device */

/* Create a context on HIP device `device`.  `hbm_budget_bytes` bounds the device memory
 * held by resident surfaces and in-flight serving requests (0 = 90% of the free memory at
 * creation).  One-shot sl_eval calls allocate their workspace stream-ordered and are not
 * counted against the budget; they take it from a memory pool of the context, which keeps what
 * it has allocated (at most the largest workspaces in use at once) until sl_destroy, so that
 * repeated calls allocate nothing new.  Returns SL_EINVAL for a bad device or NULL `out`. */
sl_status sl_create(int device, size_t hbm_budget_bytes, sl_ctx **out);

/* Drain the serving queue, stop its persistent kernel and free everything the context owns
 * (it first waits for all work on the device, which may still use pool workspaces).  NULL is a
 * no-op. */
void sl_destroy(sl_ctx *ctx);

/* Message describing the last failure on the calling thread ("" if none), whatever the
 * context; `ctx` may be NULL (failures of sl_create have none).  The pointer is valid until
 * the next library call on that thread. */
const char *sl_last_error(const sl_ctx *ctx);

/* Tunables.
 * SL_PARAM_RHO64: in SL_MIXED, pairs with r/delta below this value are summed in double
 *   precision (finite, >= 0; default 0: no such pairs).  Serving requests take the value current at
 *   sl_submit.
 * SL_PARAM_KERNEL_TIMING: 1 = bracket every pair-kernel launch of sl_eval with HIP events on
 *   the caller's stream and accumulate the elapsed time into sl_stats; 0 (default) = off.
 * SL_PARAM_TARGETS_PER_LANE: targets each lane of the pair kernels keeps in registers
 *   (1, 2 or 4; 0 = automatic, the default: 1 in SL_MIXED; in SL_FP64 1 up to 2^17 targets,
 *   2 beyond).
 * SL_PARAM_WAVES_PER_SIMD: granularity of the pair kernels' work items: the sources are split
 *   until there are about this many items per SIMD, into at most 128 ways per target block (64
 *   in SL_MIXED) (1..256; default 128). */
typedef enum {
    SL_PARAM_RHO64 = 0,
    SL_PARAM_KERNEL_TIMING = 1,
    SL_PARAM_TARGETS_PER_LANE = 2,
    SL_PARAM_WAVES_PER_SIMD = 3
} sl_param;
sl_status sl_set_param(sl_ctx *ctx, sl_param key, double value);
sl_status sl_get_param(const sl_ctx *ctx, sl_param key, double *value);

/*
 * One-shot evaluation, asynchronous on `stream` (a hipStream_t; NULL = the null stream).
 *
 *  sources:  n_src >= 0 nodes sx, sy, sz; quadrature weights w (Sec. 3.3: psi W h^2);
 *            density fx, fy, fz.
 *  targets:  n_tgt >= 0 points tx, ty, tz.  tx == ty == tz == NULL means targets = sources
 *            (then n_tgt must equal n_src).
 *  delta:    regularization length (> 0, finite) used for every target when delta_tgt is NULL;
 *            otherwise delta_tgt[n_tgt] gives one value per target (each > 0 and finite; not
 *            checked on the device -- a non-positive entry yields NaN for that target) and
 *            `delta` is ignored.
 *  mu:       viscosity (> 0, finite).
 *  output:   ux, uy, uz[n_tgt] (overwritten).
 *
 * n_src == 0 writes zeros; n_tgt == 0 enqueues nothing.  The call enqueues a spatial sort of
 * the points, the packing of w*f, the pair kernels and the final per-target reduction; the
 * workspace is allocated and freed stream-ordered on `stream`.  Results are deterministic:
 * identical inputs give bit-identical outputs.
 */
sl_status sl_eval(sl_ctx *ctx, sl_precision prec,
                  int64_t n_src, const double *sx, const double *sy, const double *sz,
                  const double *w, const double *fx, const double *fy, const double *fz,
                  int64_t n_tgt, const double *tx, const double *ty, const double *tz,
                  double delta, const double *delta_tgt, double mu,
                  double *ux, double *uy, double *uz, void *stream);

/*
 * sl_eval for callers that cannot allocate device memory (code under stream capture, serving
 * loops that must not call the allocator, harnesses that forbid allocation).  Same arguments,
 * results and errors as sl_eval, within its tolerance (the work may be split into fewer, larger
 * items so that it fits), with one difference: the workspace is a library-owned device array of
 * 256 MiB, one per GPU, held from this entry point's first call on that GPU until the process
 * ends.  The call allocates and frees nothing.  SL_EINVAL, with nothing enqueued, when a problem's
 * workspace does not fit that array even as a single work item per target block (about a million
 * points in SL_MIXED with targets = sources).  SL_PARAM_KERNEL_TIMING is ignored here.
 *
 * Every call on a GPU uses that GPU's one array: calls on one GPU must not overlap -- enqueue them
 * on one stream, or order them yourself; calls on different streams that run at the same time
 * race on the array and corrupt each other's results.  The array keeps the last call's contents;
 * each call initializes what it reads.
 */
sl_status sl_eval_noalloc(sl_ctx *ctx, sl_precision prec,
                          int64_t n_src, const double *sx, const double *sy, const double *sz,
                          const double *w, const double *fx, const double *fy, const double *fz,
                          int64_t n_tgt, const double *tx, const double *ty, const double *tz,
                          double delta, const double *delta_tgt, double mu,
                          double *ux, double *uy, double *uz, void *stream);

/*
 * Per-patch regularization parameter of Sec. 3.4, eq. (regparam), asynchronous on `stream`:
 *
 *   delta_out[p] = C delta*_i for every node p of patch i, where delta*_i is the largest
 *   Euclidean distance between two nodes of patch i that are adjacent in its grid (row,
 *   column or diagonal neighbours; an edge node has only the neighbours the grid holds).
 *
 *  x, y, z:    device arrays of n_patches n^2 nodes, patch-major and row-major within a patch
 *              (the node order of the six-patch discretization, Sec. 3.2).
 *  n_patches:  >= 1 (six for a closed surface); n >= 2 nodes per patch direction.
 *  C:          the constant of eq. (regparam) (> 0, finite; the paper takes 1).
 *  delta_out:  device array of n_patches n^2 doubles, overwritten; it must not overlap x, y, z.
 *              Pass it as delta_tgt to sl_eval (targets = the same nodes).
 *
 * The result equals a plain double loop over the definition bit for bit (squared distances
 * as ((dx dx + dy dy) + dz dz), maximum before the square root).  SL_EINVAL for bad sizes,
 * C, NULL or overlapping arrays; SL_EHIP if the launch fails.
 */
sl_status sl_patch_delta(sl_ctx *ctx, int64_t n_patches, int64_t n, const double *x,
                         const double *y, const double *z, double C, double *delta_out,
                         void *stream);

/*
 * The upsampling step of Sec. 3.4 around the sum (the upsampling, single-layer and downsampling
 * steps of the right-hand-side algorithm of Sec. 3.6), asynchronous on `stream`:
 *
 *   u = I_d S^{delta_u}[I_u f], evaluated on the upsampled surface X_u = I_u X.
 *
 *  x, y, z:     device arrays of the n_patches n^2 nodes (patch-major, row-major within a patch;
 *               a patch's nodes sit at parameters (j, k) pi / (n + 1), j, k = 1..n).
 *  W:           the area element |X_u x X_v| at the nodes (n_patches n^2, same order), as the
 *               caller computes it for the coarse weights psi W h^2 (Sec. 3.3).
 *  psi_up:      the own-patch POU value of every fine node (n_patches (factor n)^2, same order),
 *               precomputed by the caller like the POU of the coarse nodes.
 *  fx, fy, fz:  density at the nodes.
 *  factor:      fine nodes per coarse node and direction (1..8; the paper uses 4), at parameters
 *               j pi / (factor n + 1), j = 1..factor n.
 *  C, mu:       constant of eq. (regparam) for delta_u (> 0; the paper takes 1); viscosity (> 0).
 *  ux, uy, uz:  output at the nodes (n_patches n^2 each).
 *
 * I_u and I_d are per-patch tensor-product cubic splines with not-a-knot ends (the end pieces
 * extended where the fine grid reaches past the outermost nodes).  Nodes, density and area
 * element are upsampled by the same operator (X_u = I_u X, F_u = I_u F, W_u = I_u W), the fine
 * weights are psi_u W_u h_u^2 with h_u = pi / (factor n + 1), and delta_u = C delta* of the fine
 * grid (as sl_patch_delta).  The sum runs as sl_eval with targets = the fine nodes.  n >= 4 (the
 * not-a-knot spline needs four nodes).  The spline operators are built once per (n, factor) and
 * kept by the context (the first call for a size synchronizes to upload them); the rest of the
 * work is enqueued, with a workspace allocated and freed stream-ordered.  SL_EINVAL for bad sizes
 * or scalars or NULL arrays, SL_ENOMEM / SL_EHIP on allocation or launch failures.
 */
sl_status sl_eval_upsampled(sl_ctx *ctx, sl_precision prec, int64_t n_patches, int64_t n, int factor,
                            const double *x, const double *y, const double *z, const double *W,
                            const double *psi_up, const double *fx, const double *fy, const double *fz,
                            double C, double mu, double *ux, double *uy, double *uz, void *stream);

/*
 * The single layer by the single-level kernel-independent FMM of Sec. 5 ("Fast multipole method
 * based acceleration"), targets = sources, asynchronous on `stream` after a synchronization in the
 * middle (see below):
 *
 *   1. k-means clustering of the n points into k clusters (the paper takes k = 100): Lloyd's
 *      iteration from the points at indices floor(j n / k), nearest centroid by squared distance
 *      (ties to the lower index), exact centroid sums of the coordinates quantized to 2^-24 of the
 *      points' extent; it stops at the first assignment that changes no label or after max_iter
 *      assignments;
 *   2. per cluster, a cube of half width a (the box of its points' bounding box, half its largest
 *      side) with equivalent sources on the lattice of p_edge points per edge on the boundary of
 *      the cube of half width 1.05 a (N_eq = p^3 - (p - 2)^3 points), whose densities are fitted
 *      (Tikhonov least squares, weight 1e-8) to the plain-Stokeslet potential of the cluster's own
 *      points at the same lattice on the check cube of half width 2.95 a;
 *   3. per target, the regularized sum over the points of near clusters and the plain Stokeslet
 *      sum over the equivalent sources of far clusters: cluster S is far from cluster T when T's
 *      box lies outside the cube of half width 3 a_S around S's centre and at least 6.9 delta_T
 *      from S's box (delta_T the largest delta of T's points), where the smoothing factors equal 1.
 *
 *  x, y, z, w, fx, fy, fz:  the n points, weights and density (device arrays, as sl_eval).
 *  delta, delta_tgt:         as sl_eval (one delta, or one per point).
 *  k:                        clusters (1..min(n, 1024)); p_edge: 3..12; max_iter: 1..10000.
 *  ux, uy, uz:               output at the points (n each).
 *  labels_out:               NULL, or n int32: the cluster of each point.
 *
 * The result approximates sl_eval's; the error falls with p_edge (about 1e-4 relative at p = 4 to
 * 1e-7 at p = 8 on the surfaces of the paper's shape family).  The call enqueues the clustering,
 * then waits for it on `stream` (the cluster boxes come back to the host, which forms the near /
 * far lists and the padded layout), then enqueues the rest; the unit box's fit operator is built
 * on the host once per p_edge and kept by the context.  Deterministic.  SL_EINVAL for bad sizes,
 * scalars, NULL or aliasing arrays; SL_ENOMEM / SL_EHIP on allocation or launch failures.
 */
sl_status sl_eval_fmm(sl_ctx *ctx, sl_precision prec, int64_t n, const double *x, const double *y,
                      const double *z, const double *w, const double *fx, const double *fy,
                      const double *fz, double delta, const double *delta_tgt, double mu, int k,
                      int p_edge, int max_iter, double *ux, double *uy, double *uz, int32_t *labels_out,
                      void *stream);

/*
 * Serving: device-resident surfaces and continuous batching.
 *
 * sl_surface_register copies n nodes (x, y, z, w: device arrays) into library-owned HBM,
 * sorts them spatially once and keeps them resident; targets are the nodes themselves and
 * delta is fixed per surface.  It is synchronous: when the serving kernel is busy it lets the
 * queued work finish first.  Admission: SL_EBUSY if the surface's footprint does not fit the
 * remaining budget, or if submitted requests are still waiting for memory.
 *
 * sl_surface_release drops the handle; its memory is returned once no submitted request on
 * it is still in flight.
 *
 * sl_submit enqueues u = S[f] on a resident surface: fx, fy, fz (density) and ux, uy, uz
 * (output) are caller device arrays of the surface's n, valid until the request completes.
 * The request's work (one item per block of 128 targets; on a surface of at least 49,152
 * points, up to eight items per block over source ranges, whose partial sums the request's
 * staging holds) joins the queue of a single persistent kernel that serves every in-flight
 * request; requests submitted while others run are interleaved with them on the device.  Each
 * request's result is bit-identical to the same request served alone.  A request is admitted at once when its staging memory fits the
 * budget, otherwise it waits (first in, first out) until memory is returned; SL_EBUSY only if
 * its staging exceeds the whole budget.
 * Thread-safe.
 *
 * sl_poll sets *done to 1 when the request's output is complete and visible to later stream
 * work and host copies, else 0.  sl_wait blocks until then or `timeout_s` seconds
 * (SL_ETIMEDOUT).  A request id is retired by the first sl_poll/sl_wait that reports it done;
 * later queries return SL_ENOTFOUND.
 */
sl_status sl_surface_register(sl_ctx *ctx, int64_t n, const double *x, const double *y,
                              const double *z, const double *w, double delta, uint64_t *handle);
sl_status sl_surface_release(sl_ctx *ctx, uint64_t handle);
sl_status sl_submit(sl_ctx *ctx, uint64_t handle, sl_precision prec,
                    const double *fx, const double *fy, const double *fz, double mu,
                    double *ux, double *uy, double *uz, uint64_t *request);
sl_status sl_poll(sl_ctx *ctx, uint64_t request, int *done);
/* Device memory a request on surface `handle` holds from admission to completion (its staging:
 * the packed density, and for a surface large enough for split work items their partial sums,
 * at most 64 MiB), so that a client managing its own budget can make room before submitting.  SL_ENOTFOUND for an
 * unknown or released handle. */
sl_status sl_request_bytes(sl_ctx *ctx, uint64_t handle, sl_precision prec, uint64_t *bytes);
sl_status sl_wait(sl_ctx *ctx, uint64_t request, double timeout_s);

/* Statistics since sl_create (for reporting): serving requests completed, work items
 * executed, persistent-kernel launches, bytes currently admitted; and, while
 * SL_PARAM_KERNEL_TIMING is on, the number of timed sl_eval pair-kernel launches and their
 * summed duration.  Waits for the timed launches to finish. */
typedef struct {
    uint64_t requests_done;
    uint64_t items_done;
    uint64_t kernel_launches;
    uint64_t bytes_admitted;
    uint64_t pair_launches;
    double pair_ms;       /* summed duration of the timed pair-kernel launches */
} sl_stats;
sl_status sl_get_stats(sl_ctx *ctx, sl_stats *out);

#ifdef __cplusplus
}
#endif
#endif /* STOKESLET_H */
