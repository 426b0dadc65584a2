// sl_serve.hip -- resident surfaces and the continuously batched persistent kernel.
//
// Design.
//  * One HBM arena (the context's budget) holds every resident surface and the staging of every
//    admitted request.  Admission = the request's staging fits in the arena (and a descriptor
//    slot and ring space are free); requests that do not fit wait in FIFO order on the host and
//    are admitted as memory is returned.  Nothing is hipMalloc'ed or hipFree'd while the
//    persistent kernel runs (a free can synchronize the device).
//  * Work items live in a ring of host-pinned, fine-grained memory: (slot, kind, a, b).
//    kind GATHER packs g = w f for points [a, b) of the request into its staging (sorted order);
//    kind PAIR sums every source of the surface for target block a (128 targets) and writes
//    u = S[f] for those targets; on a large surface, piece b of P sums the source clusters
//    [b n / P, (b + 1) n / P) into the request's staging and the block's last piece adds the P
//    partial sums in piece order and writes u.  A request is published as its gather items
//    followed by its pair items; pair items wait for the request's gathers (which were claimed earlier, so the
//    wait is bounded).  The request's first gather item copies its descriptor from host memory
//    into device memory, where the pair items read it (one PCIe read per item instead of ~30).
//  * One persistent kernel serves all requests: each wavefront claims the next item with a CAS
//    on a device counter, runs it and counts it done; the wave finishing a request's last item
//    publishes the request's sequence number to host memory with a system-scope release.
//    The waves of a launch exit together, once the ring is drained and either the host asked
//    them to stop or no item was claimed for kIdleSeconds while none was running (the first wave
//    to see this marks the launch as exiting, and no wave claims after that mark); the host
//    relaunches the kernel when new work arrives.  The only other wait (a pair item waiting for
//    its request's gathers) is bounded as well.
//  * Coherence: staging and surfaces are reused arena memory written while the kernel runs, so
//    the kernel reads them only with vector loads after an acquire (never through the scalar
//    cache, which is only invalidated at kernel launch); each lane loads one source of a
//    cluster into the wave's own LDS area, and the source loop reads each record back at one
//    address across the wave (an LDS broadcast), so the arithmetic takes it as a vector operand.
//  * Each target's sum runs in a fixed order (clusters ascending, one accumulator set per piece,
//    the pieces added in order) whatever else is in flight, so a request's result is
//    bit-identical alone and in any mix.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <map>
#include <unordered_set>

#include "sl_internal.h"

namespace sl {

namespace {

constexpr int kServeR = 2;                       // targets per lane in a pair item
constexpr int kServeBlock = kWave * kServeR;     // targets per pair item
constexpr int64_t kGatherChunk = 4096;           // points per gather item
constexpr int kMaxSlots = 1024;                  // admitted requests in flight
constexpr uint64_t kRingCap = 1ull << 21;        // work items in the ring (power of two)
constexpr int kServeWavesPerSimd = 4;
constexpr int kServeWaves = 4;                     // waves per workgroup (one smoothing table)
// The persistent kernel exits after this idle time.  While it runs it holds every wave slot, so
// other work on the device (sl_eval, registrations) waits for it: short, while a relaunch costs
// only a launch.
constexpr double kIdleSeconds = 0.02;
constexpr double kGatherWaitSeconds = 2.0;       // bound on a pair item's wait for its gathers
constexpr double kPollSeconds = 2e-6;            // spacing of the waves' host-memory polls
constexpr double kRegisterWaitSeconds = 0.005;   // a registration's packing beside a busy kernel
// Pair items of large requests are split over source ranges: one piece per kPieceClusters source
// clusters, at most kMaxPieces, so that no item holds a wave for long.  Each piece keeps its
// partial sums (24 B per target) in the request's staging, at most kSplitBytes in all, and the
// last piece of a target block to finish adds them in piece order.
constexpr int64_t kPieceClusters = 384;
constexpr int64_t kMaxPieces = 8;
constexpr int64_t kSplitBytes = 64ll << 20;

enum : uint32_t { kItemGather = 0, kItemPair = 1 };

struct WorkItem {
    uint32_t slot, kind, a, b;
};

// Per-request descriptor in host-pinned memory (device reads it with uncached loads).
struct ReqDesc {
    const double *x, *y, *z, *w;          // surface, sorted
    const float *x32, *y32, *z32;
    const int32_t *perm;
    const double4 *sphere;
    const TBlockRec *tbr;
    const double *fx, *fy, *fz;           // caller density (caller order)
    double *ux, *uy, *uz;                 // caller output (caller order)
    double *gx, *gy, *gz;                 // staging, sorted
    float *gx32, *gy32, *gz32;
    int64_t n, np;
    double delta, scale;
    uint64_t gather_target, items_target, seq;
    int64_t mixed;
    double rho64;                         // mixed: double-precision zone p < rho64
    int64_t pieces;                       // pieces per target block (1: not split)
    double *part;                         // pieces > 1: [pieces][3][np] partial sums (staging)
    uint32_t *bdone;                      // pieces > 1: [np / 128] pieces done per target block
};

struct ServeCtl {                         // host-pinned
    uint64_t tail;                        // items published (host writes)
    uint64_t stop;                        // 1: drain and exit
    uint64_t claimed;                     // device mirror of the claim counter (lower bound)
    uint64_t error;                       // device sets 1 if a bounded wait gave up
};

struct DevCounters {                      // device memory
    uint64_t head;                        // items claimed
    uint64_t last_activity;               // wall clock of the latest claim
    uint64_t tail_mirror;                 // latest host tail seen by any wave
    uint64_t stop_mirror;                 // launch id of a wave that saw the host's stop flag
    uint64_t last_poll;                   // wall clock of the latest read of host memory
    uint64_t exit_launch;                 // id of a launch whose waves are to exit once the
                                          // queue is empty (set by the first wave to see the
                                          // stop flag or the idle limit)
    uint64_t running;                     // items claimed and not yet finished
    uint64_t pad[1];
    uint64_t gathers_done[kMaxSlots];     // monotonic per slot
    uint64_t items_done[kMaxSlots];       // monotonic per slot
};

struct ServeArgs {
    ServeCtl *ctl;
    const WorkItem *ring;
    const ReqDesc *desc;
    ReqDesc *ddesc;                       // device copies of the descriptors (written by the
                                          // request's first gather item)
    uint64_t *done_seq;                   // host-pinned, per slot
    DevCounters *dc;
    uint64_t idle_ticks;                  // exit after this long without a claim
    uint64_t wait_ticks;                  // longest wait of a pair item for its gathers
    uint64_t poll_ticks;                  // spacing of the host-memory polls
    uint64_t launch_id;                   // distinct for every launch
};

// ------------------------------------------------------------------------------------------
// Device helpers
// ------------------------------------------------------------------------------------------
__device__ __forceinline__ uint64_t ld_sys(const void *p)
{
    return __hip_atomic_load((uint64_t *)p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
}
// Doubles loaded and stored coherently across the XCDs (system scope: no stale L2 line, no
// cache maintenance).
__device__ __forceinline__ double ld_sys_f64(const double *p)
{
    return __longlong_as_double((long long)ld_sys(p));
}
__device__ __forceinline__ void st_sys_f64(double *p, double v)
{
    __hip_atomic_store((uint64_t *)p, (uint64_t)__double_as_longlong(v), __ATOMIC_RELAXED,
                       __HIP_MEMORY_SCOPE_SYSTEM);
}
__device__ __forceinline__ uint64_t uni64(uint64_t v)
{
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
    return ((uint64_t)hi << 32) | lo;
}
// A field of a descriptor's device copy, read with a vector load (never through the scalar
// cache: descriptor slots are reused while the kernel runs) and made wave-uniform.
template <typename T>
__device__ __forceinline__ T dfield(const T *p)
{
    static_assert(sizeof(T) == 8, "64-bit fields only");
    const uint64_t v = uni64(__hip_atomic_load((uint64_t *)p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
    T out;
    memcpy(&out, &v, 8);
    return out;
}
// A descriptor field, read by every lane from host memory and made wave-uniform.
template <typename T>
__device__ __forceinline__ T field(const T *p)
{
    static_assert(sizeof(T) == 8, "64-bit fields only");
    const uint64_t v = uni64(ld_sys(p));
    T out;
    memcpy(&out, &v, 8);
    return out;
}
__device__ __forceinline__ void idle_sleep(int rounds)
{
    for (int k = 0; k < rounds; ++k) __builtin_amdgcn_s_sleep(127);
}

__device__ void run_gather(const ServeArgs &a, const WorkItem &it)
{
    const ReqDesc *d = a.desc + it.slot;
    const int32_t *perm = field(&d->perm);
    const double *w = field(&d->w);
    const double *fx = field(&d->fx), *fy = field(&d->fy), *fz = field(&d->fz);
    double *gx = field(&d->gx), *gy = field(&d->gy), *gz = field(&d->gz);
    float *gx32 = field(&d->gx32), *gy32 = field(&d->gy32), *gz32 = field(&d->gz32);
    const int64_t mixed = field(&d->mixed);
    if (it.a == 0) {   // the request's descriptor, copied once into device memory for its pair items
        static_assert(sizeof(ReqDesc) % 8 == 0, "descriptor copied in 8-byte words");
        const uint64_t *src = reinterpret_cast<const uint64_t *>(d);
        uint64_t *dst = reinterpret_cast<uint64_t *>(a.ddesc + it.slot);
        for (int k = threadIdx.x % kWave; k < (int)(sizeof(ReqDesc) / 8); k += kWave) dst[k] = ld_sys(src + k);
    }
    for (int64_t p = (int64_t)it.a + threadIdx.x % kWave; p < (int64_t)it.b; p += kWave) {
        const int32_t idx = perm[p];
        double vx = 0.0, vy = 0.0, vz = 0.0;
        if (idx >= 0) {
            const double wt = w[p];
            vx = wt * fx[idx]; vy = wt * fy[idx]; vz = wt * fz[idx];
        }
        gx[p] = vx; gy[p] = vy; gz[p] = vz;
        if (mixed) { gx32[p] = (float)vx; gy32[p] = (float)vy; gz32[p] = (float)vz; }
    }
    if (field(&d->pieces) > 1) {   // the split pair items' counters of the blocks starting here
        uint32_t *bdone = field(&d->bdone);
        for (int64_t k = (int64_t)it.a / kServeBlock + threadIdx.x % kWave; k < (int64_t)it.b / kServeBlock; k += kWave)
            bdone[k] = 0u;
    }
    __threadfence();
    if (threadIdx.x % kWave == 0)
        __hip_atomic_fetch_add(&a.dc->gathers_done[it.slot], 1ull, __ATOMIC_RELEASE,
                               __HIP_MEMORY_SCOPE_AGENT);
}

// Per-wave LDS staging of one cluster's sources: 64 double-precision records (x, y, z, gx, gy, gz,
// two spare) and 64 single-precision ones.  Each lane stores one source with coalesced loads; the
// source loop then reads every record at one address across the wave (a broadcast), so the VALU
// instructions take it as an ordinary vector operand.  A wave reads only what it wrote itself,
// and LDS operations of one wave complete in order, so no barrier is needed.
struct Stage {
    double4 *d;   // [kCluster][2]
    float4 *f;    // [kCluster][2]
};

// What a pair item reads of its request, and its target block's classification record.
struct BlockView {
    const double *sx, *sy, *sz, *gx, *gy, *gz;
    const float *sx32, *sy32, *sz32, *gx32, *gy32, *gz32;
    const int32_t *perm;
    const double4 *sphere;
    double *ux, *uy, *uz;
    int64_t np;
    int64_t c_lo, c_hi;                   // the source clusters of this item
    double *part;                         // split items: this piece's [3][np] partial sums
    double scale, gap_far;
    TBlockRec rec;
    DeltaC dc;
    DeltaC32 dc32;
};

// The sums of the R * 64 targets from t0 on over the source clusters [c_lo, c_hi) of the request,
// written to the caller's arrays (or, for a piece of a split item, unscaled to its partial sums).  MIXED: single precision with the per-cluster two-sum, and with ZONE
// the pairs below rho64 in double precision; otherwise every pair in double precision.
template <bool MIXED, bool ZONE, int R>
__device__ __forceinline__ void serve_targets(const BlockView &v, int64_t t0, const float4 *tab,
                                              const Stage &st)
{
    constexpr bool F64 = !MIXED || ZONE;   // double-precision targets and sums
    const int lane = threadIdx.x % kWave;
    double tx[F64 ? R : 1], ty[F64 ? R : 1], tz[F64 ? R : 1];
    double ax[F64 ? R : 1], ay[F64 ? R : 1], az[F64 ? R : 1];
    float tx32[MIXED ? R : 1], ty32[MIXED ? R : 1], tz32[MIXED ? R : 1];
    float hx[MIXED ? R : 1], hy[MIXED ? R : 1], hz[MIXED ? R : 1];
    float lx[MIXED ? R : 1], ly[MIXED ? R : 1], lz[MIXED ? R : 1];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int64_t i = t0 + r * kWave + lane;
        if constexpr (F64) {
            tx[r] = v.sx[i]; ty[r] = v.sy[i]; tz[r] = v.sz[i];
            ax[r] = ay[r] = az[r] = 0.0;
        }
        if constexpr (MIXED) {
            tx32[r] = v.sx32[i]; ty32[r] = v.sy32[i]; tz32[r] = v.sz32[i];
            hx[r] = hy[r] = hz[r] = lx[r] = ly[r] = lz[r] = 0.0f;
        }
    }

    for (int64_t c = v.c_lo; c < v.c_hi; ++c) {
        const int64_t j0 = c * kCluster;
        const bool far = uni64(cluster_is_far(v.rec, v.sphere[c], v.gap_far) ? 1u : 0u) != 0;
        // stage what this cluster's loop reads
        if constexpr (MIXED) {
            st.f[2 * lane] = make_float4(v.sx32[j0 + lane], v.sy32[j0 + lane], v.sz32[j0 + lane],
                                         v.gx32[j0 + lane]);
            st.f[2 * lane + 1] = make_float4(v.gy32[j0 + lane], v.gz32[j0 + lane], 0.0f, 0.0f);
        }
        if (!MIXED || (ZONE && !far)) {
            st.d[2 * lane] = make_double4(v.sx[j0 + lane], v.sy[j0 + lane], v.sz[j0 + lane],
                                          v.gx[j0 + lane]);
            st.d[2 * lane + 1] = make_double4(v.gy[j0 + lane], v.gz[j0 + lane], 0.0, 0.0);
        }
        if constexpr (MIXED) {
            float px[R], py[R], pz[R];
#pragma unroll
            for (int r = 0; r < R; ++r) px[r] = py[r] = pz[r] = 0.0f;
            if (far) {
#pragma unroll 4
                for (int j = 0; j < kCluster; ++j) {
                    const float4 u = st.f[2 * j], w = st.f[2 * j + 1];
#pragma unroll
                    for (int r = 0; r < R; ++r)
                        far_pair32(tx32[r], ty32[r], tz32[r], u.x, u.y, u.z, u.w, w.x, w.y, px[r],
                                   py[r], pz[r]);
                }
            } else {
#pragma unroll ZONE ? 1 : 2
                for (int j = 0; j < kCluster; ++j) {
                    const float4 u = st.f[2 * j], w = st.f[2 * j + 1];
                    bool z64[R], any = false;
#pragma unroll
                    for (int r = 0; r < R; ++r) {
                        near_pair32<ZONE>(tx32[r], ty32[r], tz32[r], u.x, u.y, u.z, u.w, w.x, w.y,
                                          v.dc32, tab, px[r], py[r], pz[r]);
                        if constexpr (ZONE) {
                            float ex, ey, ez;
                            z64[r] = diff32(tx32[r], ty32[r], tz32[r], u.x, u.y, u.z, ex, ey, ez) <
                                     v.dc32.cut2_64;
                            any = any || z64[r];
                        }
                    }
                    if constexpr (ZONE) {
                        if (__builtin_amdgcn_ballot_w64(any)) {
                            const double4 U = st.d[2 * j], V = st.d[2 * j + 1];
#pragma unroll
                            for (int r = 0; r < R; ++r)
                                if (z64[r])
                                    zone_pair64(tx[r], ty[r], tz[r], U.x, U.y, U.z, U.w, V.x, V.y,
                                                v.dc, ax[r], ay[r], az[r]);
                        }
                    }
                }
            }
#pragma unroll
            for (int r = 0; r < R; ++r) {
                two_sum_acc(px[r], hx[r], lx[r]);
                two_sum_acc(py[r], hy[r], ly[r]);
                two_sum_acc(pz[r], hz[r], lz[r]);
            }
        } else if (far) {
#pragma unroll 2
            for (int j = 0; j < kCluster; ++j) {
                const double4 u = st.d[2 * j], w = st.d[2 * j + 1];
#pragma unroll
                for (int r = 0; r < R; ++r)
                    far_pair64(tx[r], ty[r], tz[r], u.x, u.y, u.z, u.w, w.x, w.y, ax[r], ay[r], az[r]);
            }
        } else {
#pragma unroll 1
            for (int j = 0; j < kCluster; ++j) {
                const double4 u = st.d[2 * j], w = st.d[2 * j + 1];
#pragma unroll
                for (int r = 0; r < R; ++r)
                    near_pair64(tx[r], ty[r], tz[r], u.x, u.y, u.z, u.w, w.x, w.y, v.dc, ax[r], ay[r],
                                az[r]);
            }
        }
    }

#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int64_t i = t0 + r * kWave + lane;
        const int32_t idx = v.perm[i];
        if (idx >= 0 || v.part) {
            double ox, oy, oz;
            if constexpr (MIXED) {
                ox = (double)hx[r] + (double)lx[r];
                oy = (double)hy[r] + (double)ly[r];
                oz = (double)hz[r] + (double)lz[r];
                if constexpr (ZONE) {
                    ox = ax[r] + ox;
                    oy = ay[r] + oy;
                    oz = az[r] + oz;
                }
            } else {
                ox = ax[r];
                oy = ay[r];
                oz = az[r];
            }
            if (v.part) {
                // written through to memory (system scope, no cache maintenance): the piece that
                // adds them may run on another XCD
                st_sys_f64(v.part + i, ox);
                st_sys_f64(v.part + v.np + i, oy);
                st_sys_f64(v.part + 2 * v.np + i, oz);
            } else {
                v.ux[idx] = ox * v.scale;
                v.uy[idx] = oy * v.scale;
                v.uz[idx] = oz * v.scale;
            }
        }
    }
}

// The last piece of a split target block: the pieces' partial sums (`part`: [pieces][3][np])
// added in piece order, scaled and scattered to the caller's arrays.
__device__ void combine_pieces(const BlockView &v, const double *part, int64_t pieces, int64_t t0)
{
    const int lane = threadIdx.x % kWave;
    for (int r = 0; r < kServeR; ++r) {
        const int64_t i = t0 + r * kWave + lane;
        const int32_t idx = v.perm[i];
        if (idx < 0) continue;
        double ox = 0.0, oy = 0.0, oz = 0.0;
        for (int64_t q = 0; q < pieces; ++q) {
            const double *pq = part + q * 3 * v.np;
            ox += ld_sys_f64(pq + i);
            oy += ld_sys_f64(pq + v.np + i);
            oz += ld_sys_f64(pq + 2 * v.np + i);
        }
        v.ux[idx] = ox * v.scale;
        v.uy[idx] = oy * v.scale;
        v.uz[idx] = oz * v.scale;
    }
}

__device__ void run_pair(const ServeArgs &a, const WorkItem &it, const float4 *tab, const Stage &st)
{
    const int lane = threadIdx.x % kWave;
    const ReqDesc *d = a.desc + it.slot;
    // Wait until the request's density is packed.  Its gather items were claimed before this
    // item by running waves, so the wait ends; it is still bounded, and on expiry the item
    // reports an error to the host and completes without writing.
    const uint64_t gather_target = field(&d->gather_target);
    const uint64_t t_wait0 = wall_clock64();
    bool ready = false;
    for (int rounds = 1;; rounds = rounds < 8 ? rounds * 2 : 8) {
        uint64_t g = 0;
        if (lane == 0)
            g = __hip_atomic_load(&a.dc->gathers_done[it.slot], __ATOMIC_RELAXED,
                                  __HIP_MEMORY_SCOPE_SYSTEM);
        if (uni64(g) >= gather_target) {
            ready = true;
            break;
        }
        if (uni64(wall_clock64() - t_wait0 > a.wait_ticks ? 1u : 0u)) break;
        idle_sleep(rounds);
    }
    __atomic_thread_fence(__ATOMIC_ACQUIRE);
    if (!ready) {
        if (lane == 0) {
            __hip_atomic_store(&a.ctl->error, 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
            const uint64_t items_target = ld_sys(&d->items_target);
            const uint64_t old = __hip_atomic_fetch_add(&a.dc->items_done[it.slot], 1ull,
                                                        __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
            if (old + 1 == items_target)
                __hip_atomic_store(&a.done_seq[it.slot], ld_sys(&d->seq), __ATOMIC_RELEASE,
                                   __HIP_MEMORY_SCOPE_SYSTEM);
        }
        return;
    }

    const ReqDesc *dd = a.ddesc + it.slot;   // written before the gathers finished
    BlockView v;
    v.sx = dfield(&dd->x); v.sy = dfield(&dd->y); v.sz = dfield(&dd->z);
    v.gx = dfield(&dd->gx); v.gy = dfield(&dd->gy); v.gz = dfield(&dd->gz);
    v.sx32 = dfield(&dd->x32); v.sy32 = dfield(&dd->y32); v.sz32 = dfield(&dd->z32);
    v.gx32 = dfield(&dd->gx32); v.gy32 = dfield(&dd->gy32); v.gz32 = dfield(&dd->gz32);
    v.perm = dfield(&dd->perm);
    v.sphere = dfield(&dd->sphere);
    v.ux = dfield(&dd->ux); v.uy = dfield(&dd->uy); v.uz = dfield(&dd->uz);
    v.np = dfield(&dd->np);
    v.scale = dfield(&dd->scale);
    const double delta = dfield(&dd->delta);
    const bool mixed = dfield(&dd->mixed) != 0;
    const TBlockRec *tbr = dfield(&dd->tbr);
    v.rec = tbr[it.a];
    const double rho64 = dfield(&dd->rho64);
    // the mixed far cut of the surface (5 delta, widened for the box size) and this request's own
    // double-precision zone
    v.gap_far = mixed ? fmax(v.rec.gap_far_mixed, rho64 * delta) : v.rec.gap_far;
    v.dc = make_delta(delta);
    v.dc32 = make_delta32(delta, rho64);
    const int64_t t0 = (int64_t)it.a * kServeBlock;
    const int64_t pieces = dfield(&dd->pieces);
    const int64_t piece = it.b;
    double *const part = pieces > 1 ? dfield(&dd->part) : nullptr;
    const int64_t n_cl = v.np / kCluster;
    v.c_lo = piece * n_cl / pieces;
    v.c_hi = (piece + 1) * n_cl / pieces;
    v.part = part ? part + piece * 3 * v.np : nullptr;
    // One instance per path, so that no path holds another's registers; the mixed path with the
    // double-precision zone, whose pairs hold the most state, takes half of the targets at a time.
    if (!mixed) {
        serve_targets<false, false, kServeR>(v, t0, tab, st);
    } else if (v.dc32.cut2_64 > 0.0f) {
        for (int h = 0; h < kServeR; ++h) serve_targets<true, true, 1>(v, t0 + h * kWave, tab, st);
    } else {
        serve_targets<true, false, kServeR>(v, t0, tab, st);
    }
    bool wrote_output = true;
    if (part) {
        // The piece's partial sums were written through to memory; once the wave's stores are
        // complete it counts itself done on the block.  The last piece reads them all from
        // memory, adds them in piece order and writes the block's output.
        // The wave's write-through stores are acknowledged before the count: a wait on the
        // vector-memory counter (a workgroup-scope fence would not wait for global stores, and an
        // agent-scope one would write back the whole L2).
        asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
        uint32_t old = 0;
        if (lane == 0)
            old = __hip_atomic_fetch_add(dfield(&dd->bdone) + it.a, 1u, __ATOMIC_RELAXED,
                                         __HIP_MEMORY_SCOPE_SYSTEM);
        wrote_output = uni64(old) + 1 == (uint64_t)pieces;
        if (wrote_output) {
            // the partial sums are read after the count (they bypass the caches)
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
            combine_pieces(v, part, pieces, t0);
        }
    }
    // an item that wrote output releases it (write-back of this XCD's L2) before it counts
    if (wrote_output) __threadfence();
    if (lane == 0) {
        const uint64_t items_target = dfield(&dd->items_target);
        const uint64_t old = wrote_output
                                 ? __hip_atomic_fetch_add(&a.dc->items_done[it.slot], 1ull,
                                                          __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT)
                                 : __hip_atomic_fetch_add(&a.dc->items_done[it.slot], 1ull,
                                                          __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (old + 1 == items_target) {
            __threadfence_system();
            __hip_atomic_store(&a.done_seq[it.slot], dfield(&dd->seq), __ATOMIC_RELEASE,
                               __HIP_MEMORY_SCOPE_SYSTEM);
        }
    }
}

__global__ __launch_bounds__(kServeWaves * kWave) void k_serve(ServeArgs a)
{
    __shared__ float4 sh_tab[kTab32Rows];   // single-precision smoothing table, shared
    __shared__ double4 sh_d[kServeWaves][2 * kCluster];
    __shared__ float4 sh_f[kServeWaves][2 * kCluster];
    load_tab32(sh_tab);
    __syncthreads();
    // From here on every wave works on its own: it pulls its own items and leaves on its own.
    const int lane = threadIdx.x % kWave, wv = threadIdx.x / kWave;
    const Stage stage{sh_d[wv], sh_f[wv]};
    // The idle clock of this wave starts no earlier than the wave itself: the shared activity
    // time may still hold the previous launch's last claim, and a wave that read it would take
    // the new launch for idle.  The stop and exit marks carry the launch id for the same reason.
    const uint64_t t_start = uni64(wall_clock64());
    int rounds = 0;
    for (;;) {
        uint64_t idx = 0, got = 0, quit = 0, w0 = 0, w1 = 0;
        if (lane == 0) {
            // Polling loads at system scope: coherent across the XCDs' L2 caches without any
            // cache maintenance (agent-scope relaxed loads may hit a stale line in this XCD's L2,
            // and agent-scope acquires would invalidate the whole L2).
            uint64_t h = __hip_atomic_load(&a.dc->head, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
            uint64_t t = __hip_atomic_load(&a.dc->tail_mirror, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
            // Once this launch is exiting, no wave takes new work: items published meanwhile
            // wait for the relaunch.  (A few waves left claiming would keep the launch alive on
            // a fraction of the chip while requests keep coming.)
            const bool exiting = __hip_atomic_load(&a.dc->exit_launch, __ATOMIC_RELAXED,
                                                   __HIP_MEMORY_SCOPE_SYSTEM) == a.launch_id;
            if (exiting) {
                quit = 1;
            } else if (h >= t) {
                // At most one wave every ~2 us reads the host's tail and stop flag (PCIe) and
                // mirrors them into device memory for the others.
                const uint64_t now = wall_clock64();
                uint64_t lp = __hip_atomic_load(&a.dc->last_poll, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
                if (now > lp + a.poll_ticks &&
                    __hip_atomic_compare_exchange_strong(&a.dc->last_poll, &lp, now, __ATOMIC_RELAXED,
                                                         __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM)) {
                    t = __hip_atomic_load(&a.ctl->tail, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
                    const uint64_t stop = __hip_atomic_load(&a.ctl->stop, __ATOMIC_RELAXED,
                                                            __HIP_MEMORY_SCOPE_SYSTEM);
                    __hip_atomic_fetch_max(&a.dc->tail_mirror, t, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
                    if (stop)
                        __hip_atomic_store(&a.dc->stop_mirror, a.launch_id, __ATOMIC_RELAXED,
                                           __HIP_MEMORY_SCOPE_SYSTEM);
                }
            }
            if (!exiting && h < t) {
                // Read the slot before claiming it.  Claims succeed in index order, so once the
                // claim of h succeeds every item below h + 1 has been read, and any claim count
                // published afterwards is a lower bound of the items read: the host never reuses
                // a slot that a wave has claimed but not yet read.  (If the claim fails, the
                // values are dropped.)
                const WorkItem *slot = a.ring + (h & (kRingCap - 1));
                const uint64_t v0 = ld_sys(slot), v1 = ld_sys((const uint64_t *)slot + 1);
                // the slot's loads complete before the claim (a wave-local wait, no cache
                // maintenance: idle waves poll here, and an agent-scope fence per poll would
                // write back and invalidate L2 under the waves that are working)
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
                if (__hip_atomic_compare_exchange_strong(&a.dc->head, &h, h + 1, __ATOMIC_RELAXED,
                                                         __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM)) {
                    got = 1;
                    idx = h;
                    w0 = v0;
                    w1 = v1;
                    __hip_atomic_fetch_add(&a.dc->running, 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
                }
            } else if (!exiting) {
                const bool stop = __hip_atomic_load(&a.dc->stop_mirror, __ATOMIC_RELAXED,
                                                    __HIP_MEMORY_SCOPE_SYSTEM) == a.launch_id;
                uint64_t last = __hip_atomic_load(&a.dc->last_activity, __ATOMIC_RELAXED,
                                                  __HIP_MEMORY_SCOPE_SYSTEM);
                last = last > t_start ? last : t_start;
                const uint64_t now = wall_clock64();
                const uint64_t running = __hip_atomic_load(&a.dc->running, __ATOMIC_RELAXED,
                                                           __HIP_MEMORY_SCOPE_SYSTEM);
                // All waves of a launch exit together, on the host's stop flag once the queue is
                // empty, or when nothing has been claimed for the idle limit and nothing runs.
                if (stop || (running == 0 && now > last && now - last > a.idle_ticks)) {
                    __hip_atomic_store(&a.dc->exit_launch, a.launch_id, __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_SYSTEM);
                    quit = 1;
                }
            }
        }
        got = uni64(got);
        if (!got) {
            if (uni64(quit)) break;
            rounds = rounds < 16 ? rounds + 1 : 16;
            idle_sleep(rounds);
            continue;
        }
        rounds = 0;
        idx = uni64(idx);
        if (lane == 0) {
            __hip_atomic_fetch_max(&a.dc->last_activity, (uint64_t)wall_clock64(), __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_SYSTEM);
            // claim count for the host's ring-space check: every item below it has been read
            // (plain store: out-of-order writers can only make it smaller, which is safe)
            __hip_atomic_store(&a.ctl->claimed, idx + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
        }
        w0 = uni64(w0);
        w1 = uni64(w1);
        WorkItem it;
        it.slot = (uint32_t)w0;
        it.kind = (uint32_t)(w0 >> 32);
        it.a = (uint32_t)w1;
        it.b = (uint32_t)(w1 >> 32);
        __atomic_thread_fence(__ATOMIC_ACQUIRE);
        if (it.kind == kItemGather)
            run_gather(a, it);
        else
            run_pair(a, it, sh_tab, stage);
        if (lane == 0)
            __hip_atomic_fetch_add(&a.dc->running, ~0ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
    }
}

// Surface packing at registration: sorted positions and weights, single-precision positions,
// permutation, cluster spheres.
__global__ __launch_bounds__(256) void k_gather_surface(
    const uint32_t *__restrict__ order, int64_t n, const double *__restrict__ x,
    const double *__restrict__ y, const double *__restrict__ z, const double *__restrict__ w,
    const double *__restrict__ centre, double *ox, double *oy, double *oz, double *ow, float *ox32,
    float *oy32, float *oz32, int32_t *operm, double4 *osphere)
{
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const bool real = p < n;
    const uint32_t idx = order[real ? p : n - 1];
    const double px = x[idx], py = y[idx], pz = z[idx];
    ox[p] = px; oy[p] = py; oz[p] = pz;
    ow[p] = real ? w[idx] : 0.0;
    ox32[p] = (float)(px - centre[0]);
    oy32[p] = (float)(py - centre[1]);
    oz32[p] = (float)(pz - centre[2]);
    operm[p] = real ? (int32_t)idx : -1;
    const double cx = 0.5 * (wave_min(px) + wave_max(px));
    const double cy = 0.5 * (wave_min(py) + wave_max(py));
    const double cz = 0.5 * (wave_min(pz) + wave_max(pz));
    const double dx = px - cx, dy = py - cy, dz = pz - cz;
    const double rad = sqrt(wave_max(fma(dx, dx, fma(dy, dy, __dmul_rn(dz, dz))))) * (1.0 + 0x1p-40);
    if ((threadIdx.x % kWave) == 0) osphere[p / kCluster] = make_double4(cx, cy, cz, rad);
}

// Target-block records for pair items, with the far thresholds of both precisions (the mixed one
// without any double-precision zone: a request widens it by its own rho64).
__global__ __launch_bounds__(kWave) void k_tblock_serve(const double *__restrict__ x,
                                                        const double *__restrict__ y,
                                                        const double *__restrict__ z,
                                                        const double *__restrict__ bbox,
                                                        double delta, TBlockRec *__restrict__ out)
{
    const int tb = blockIdx.x, lane = threadIdx.x;
    double px[kServeR], py[kServeR], pz[kServeR];
    double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
#pragma unroll
    for (int r = 0; r < kServeR; ++r) {
        const int64_t i = (int64_t)tb * kServeBlock + r * kWave + lane;
        px[r] = x[i]; py[r] = y[i]; pz[r] = z[i];
        lo[0] = fmin(lo[0], px[r]); hi[0] = fmax(hi[0], px[r]);
        lo[1] = fmin(lo[1], py[r]); hi[1] = fmax(hi[1], py[r]);
        lo[2] = fmin(lo[2], pz[r]); hi[2] = fmax(hi[2], pz[r]);
    }
    const double cx = 0.5 * (wave_min(lo[0]) + wave_max(hi[0]));
    const double cy = 0.5 * (wave_min(lo[1]) + wave_max(hi[1]));
    const double cz = 0.5 * (wave_min(lo[2]) + wave_max(hi[2]));
    double rr = 0.0;
#pragma unroll
    for (int r = 0; r < kServeR; ++r) {
        const double dx = px[r] - cx, dy = py[r] - cy, dz = pz[r] - cz;
        rr = fmax(rr, fma(dx, dx, fma(dy, dy, __dmul_rn(dz, dz))));
    }
    rr = wave_max(rr);
    if (lane == 0) {
        const double bx = bbox[3] - bbox[0], by = bbox[4] - bbox[1], bz = bbox[5] - bbox[2];
        TBlockRec rec;
        rec.cx = cx; rec.cy = cy; rec.cz = cz;
        rec.rad = sqrt(rr) * (1.0 + 0x1p-40);
        rec.gap_far = kRhoExact64 * delta;
        rec.gap_far_mixed = fmax(kRhoExact32 * delta,
                                 0x1p-10 * sqrt(fma(bx, bx, fma(by, by, __dmul_rn(bz, bz)))));
        rec.pad0 = rec.pad1 = 0.0;
        out[tb] = rec;
    }
}

// ------------------------------------------------------------------------------------------
// Host side
// ------------------------------------------------------------------------------------------
// First-fit allocator over one device buffer (offsets aligned to 256 bytes).
class Arena {
public:
    char *base = nullptr;
    size_t size = 0, used = 0;

    void init(char *b, size_t s)
    {
        base = b;
        size = s;
        free_[0] = s;
    }
    char *alloc(size_t bytes)
    {
        bytes = (size_t)round_up((int64_t)bytes, 256);
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= bytes) {
                const size_t off = it->first, len = it->second;
                free_.erase(it);
                if (len > bytes) free_[off + bytes] = len - bytes;
                used += bytes;
                sizes_[off] = bytes;
                return base + off;
            }
        }
        return nullptr;
    }
    // The block at p of `bytes` (p inside a free block that holds it): undoes a release.
    char *alloc_at(char *p, size_t bytes)
    {
        bytes = (size_t)round_up((int64_t)bytes, 256);
        const size_t off = (size_t)(p - base);
        auto it = free_.upper_bound(off);
        if (it == free_.begin()) return nullptr;
        --it;
        const size_t fo = it->first, fl = it->second;
        if (off < fo || off + bytes > fo + fl) return nullptr;
        free_.erase(it);
        if (off > fo) free_[fo] = off - fo;
        if (off + bytes < fo + fl) free_[off + bytes] = fo + fl - off - bytes;
        used += bytes;
        sizes_[off] = bytes;
        return p;
    }
    void release(char *p)
    {
        const size_t off = (size_t)(p - base);
        auto s = sizes_.find(off);
        if (s == sizes_.end()) return;
        size_t len = s->second;
        sizes_.erase(s);
        used -= len;
        size_t start = off;
        auto next = free_.lower_bound(off);
        if (next != free_.end() && next->first == off + len) {
            len += next->second;
            free_.erase(next);
        }
        auto prev = free_.lower_bound(off);
        if (prev != free_.begin()) {
            --prev;
            if (prev->first + prev->second == off) {
                start = prev->first;
                len += prev->second;
                free_.erase(prev);
            }
        }
        free_[start] = len;
    }

private:
    std::map<size_t, size_t> free_;    // offset -> length
    std::map<size_t, size_t> sizes_;   // offset -> length of live blocks
};

struct Surface {
    int64_t n = 0, np = 0;
    double delta = 0.0;
    char *mem = nullptr;
    double *x, *y, *z, *w;
    float *x32, *y32, *z32;
    int32_t *perm;
    double4 *sphere;
    TBlockRec *tbr;
    int refs = 0;
    bool released = false;
};

// The arrays of a resident surface inside its arena block (as written by the registration).
void surface_layout(Surface &sf, char *mem)
{
    const int64_t np = sf.np;
    sf.mem = mem;
    char *p = mem;
    auto take = [&](int64_t bytes) { char *q = p; p += round_up(bytes, 256); return q; };
    sf.x = (double *)take(np * 8); sf.y = (double *)take(np * 8); sf.z = (double *)take(np * 8);
    sf.w = (double *)take(np * 8);
    sf.x32 = (float *)take(np * 4); sf.y32 = (float *)take(np * 4); sf.z32 = (float *)take(np * 4);
    sf.perm = (int32_t *)take(np * 4);
    sf.sphere = (double4 *)take(np / kCluster * (int64_t)sizeof(double4));
    sf.tbr = (TBlockRec *)take(np / kServeBlock * (int64_t)sizeof(TBlockRec));
}

enum class ReqState { Pending, Active, Done, Failed };

struct HostReq {
    uint64_t id = 0;
    uint64_t surf = 0;
    bool mixed = false;
    const double *fx, *fy, *fz;
    double *ux, *uy, *uz;
    double mu = 1.0;
    double rho64 = 0.0;
    ReqState state = ReqState::Pending;
    int slot = -1;
    char *staging = nullptr;
    uint64_t seq = 0;
    uint64_t n_items = 0;
};

}  // namespace

struct Server {
    sl_ctx *ctx = nullptr;
    std::mutex mu;
    std::condition_variable cv;          // progress thread wake-up
    std::condition_variable done_cv;     // waiters
    std::thread thread;
    bool quit = false;
    sl_status fatal = SL_OK;
    std::string fatal_msg;

    Arena arena;
    char *arena_mem = nullptr;
    hipStream_t kstream = nullptr, aux = nullptr;
    hipEvent_t kdone = nullptr;
    double clock_hz = 100e6;             // rate of the device's constant wall clock
    bool kernel_launched = false;
    int registering = 0;                 // registrations in progress: no kernel relaunch meanwhile

    ServeCtl *ctl = nullptr;
    WorkItem *ring = nullptr;
    ReqDesc *desc = nullptr;
    uint64_t *done_seq = nullptr;
    DevCounters *dc = nullptr;
    ReqDesc *ddesc = nullptr;             // device copies of the descriptors
    uint64_t gathers_cum[kMaxSlots] = {};
    uint64_t items_cum[kMaxSlots] = {};
    std::vector<int> free_slots;

    std::unordered_map<uint64_t, Surface> surfaces;
    std::unordered_map<uint64_t, HostReq> reqs;
    std::deque<uint64_t> pending;
    std::vector<uint64_t> active;
    uint64_t next_surface = 1, next_req = 1, next_seq = 1;
    uint64_t tail = 0;
    sl_stats stats = {};

    sl_status init(sl_ctx *c);
    void shutdown();
    void loop();
    void complete_locked();
    void admit_locked();
    bool compact_locked();
    sl_status ensure_kernel_locked();
    void free_surface_locked(uint64_t h);
};

namespace {

size_t surface_bytes(int64_t np)
{
    const int64_t nb = np / kServeBlock;
    return (size_t)(4 * round_up(np * 8, 256) + 3 * round_up(np * 4, 256) + round_up(np * 4, 256) +
                    round_up(np / kCluster * (int64_t)sizeof(double4), 256) +
                    round_up(nb * (int64_t)sizeof(TBlockRec), 256));
}

int64_t pieces_for(int64_t np)
{
    int64_t p = np / kCluster / kPieceClusters;
    p = p > kMaxPieces ? kMaxPieces : p;
    while (p > 1 && p * 3 * np * 8 > kSplitBytes) --p;
    return p < 1 ? 1 : p;
}

size_t staging_bytes(int64_t np, bool mixed)
{
    const int64_t pieces = pieces_for(np);
    return (size_t)(3 * round_up(np * 8, 256) + (mixed ? 3 * round_up(np * 4, 256) : 0) +
                    (pieces > 1 ? round_up(pieces * 3 * np * 8, 256) + round_up(np / kServeBlock * 4, 256) : 0));
}

}  // namespace

sl_status Server::init(sl_ctx *c)
{
    ctx = c;
    SL_HIP(hipStreamCreateWithFlags(&kstream, hipStreamNonBlocking));
    SL_HIP(hipStreamCreateWithFlags(&aux, hipStreamNonBlocking));
    SL_HIP(hipEventCreateWithFlags(&kdone, hipEventDisableTiming));
    int khz = 0;
    if (hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, ctx->device) == hipSuccess && khz > 0)
        clock_hz = 1e3 * (double)khz;
    SL_HIP(hipHostMalloc((void **)&ctl, sizeof(ServeCtl), hipHostMallocCoherent | hipHostMallocMapped));
    SL_HIP(hipHostMalloc((void **)&ring, sizeof(WorkItem) * kRingCap, hipHostMallocCoherent | hipHostMallocMapped));
    SL_HIP(hipHostMalloc((void **)&desc, sizeof(ReqDesc) * kMaxSlots, hipHostMallocCoherent | hipHostMallocMapped));
    SL_HIP(hipHostMalloc((void **)&done_seq, sizeof(uint64_t) * kMaxSlots, hipHostMallocCoherent | hipHostMallocMapped));
    memset((void *)ctl, 0, sizeof(ServeCtl));
    memset((void *)desc, 0, sizeof(ReqDesc) * kMaxSlots);
    memset((void *)done_seq, 0, sizeof(uint64_t) * kMaxSlots);
    SL_HIP(hipMalloc((void **)&dc, sizeof(DevCounters)));
    SL_HIP(hipMalloc((void **)&ddesc, sizeof(ReqDesc) * kMaxSlots));
    SL_HIP(hipMemsetAsync(dc, 0, sizeof(DevCounters), aux));
    size_t bytes = ctx->budget;
    SL_HIP(hipMalloc((void **)&arena_mem, bytes));
    SL_HIP(hipStreamSynchronize(aux));
    arena.init(arena_mem, bytes);
    for (int s = kMaxSlots - 1; s >= 0; --s) free_slots.push_back(s);
    thread = std::thread([this] { loop(); });
    return SL_OK;
}

void Server::shutdown()
{
    {
        std::unique_lock<std::mutex> l(mu);
        quit = true;
    }
    cv.notify_all();
    if (thread.joinable()) thread.join();
    // Drain: the kernel processes every published item, then sees `stop` and exits.
    __atomic_store_n(&ctl->stop, 1ull, __ATOMIC_RELEASE);
    if (kstream) (void)hipStreamSynchronize(kstream);
    if (aux) (void)hipStreamSynchronize(aux);
    if (arena_mem) (void)hipFree(arena_mem);
    if (dc) (void)hipFree(dc);
    if (ddesc) (void)hipFree(ddesc);
    if (ctl) (void)hipHostFree(ctl);
    if (ring) (void)hipHostFree(ring);
    if (desc) (void)hipHostFree(desc);
    if (done_seq) (void)hipHostFree(done_seq);
    if (kdone) (void)hipEventDestroy(kdone);
    if (kstream) (void)hipStreamDestroy(kstream);
    if (aux) (void)hipStreamDestroy(aux);
}

void Server::free_surface_locked(uint64_t h)
{
    auto it = surfaces.find(h);
    if (it == surfaces.end()) return;
    arena.release(it->second.mem);
    surfaces.erase(it);
}

void Server::complete_locked()
{
    bool any = false;
    for (size_t k = 0; k < active.size();) {
        HostReq &r = reqs[active[k]];
        const uint64_t seen = __atomic_load_n(&done_seq[r.slot], __ATOMIC_ACQUIRE);
        if (seen != r.seq) {
            ++k;
            continue;
        }
        r.state = ReqState::Done;
        arena.release(r.staging);
        r.staging = nullptr;
        free_slots.push_back(r.slot);
        Surface &s = surfaces[r.surf];
        if (--s.refs == 0 && s.released) free_surface_locked(r.surf);
        stats.requests_done += 1;
        stats.items_done += r.n_items;
        active[k] = active.back();
        active.pop_back();
        any = true;
    }
    if (any) done_cv.notify_all();
}

// Moves the resident surfaces that no admitted request reads toward the start of the arena, so
// that the free bytes come together (first fit can otherwise leave a request that the free
// bytes would hold waiting for good).  Each copy goes through a scratch buffer (source and
// destination may overlap) on the auxiliary stream, and the call waits for them: surfaces of
// pending requests are not read before admission, idle ones not at all.  Returns whether
// anything moved.
bool Server::compact_locked()
{
    std::unordered_set<uint64_t> pinned;
    for (uint64_t id : active) pinned.insert(reqs[id].surf);
    std::vector<std::pair<char *, uint64_t>> order;
    for (auto &kv : surfaces)
        if (!pinned.count(kv.first)) order.emplace_back(kv.second.mem, kv.first);
    std::sort(order.begin(), order.end());
    bool moved = false;
    hipError_t e = hipSuccess;
    for (auto &o : order) {
        Surface &sf = surfaces[o.second];
        const size_t bytes = surface_bytes(sf.np);
        char *old = sf.mem;
        arena.release(old);
        char *nw = arena.alloc(bytes);   // the block just released fits, at the latest
        if (nw == old) continue;
        void *tmp = nullptr;
        e = ws_alloc(ctx, &tmp, bytes, aux);
        if (e == hipSuccess) e = hipMemcpyAsync(tmp, old, bytes, hipMemcpyDeviceToDevice, aux);
        if (e == hipSuccess) e = hipMemcpyAsync(nw, tmp, bytes, hipMemcpyDeviceToDevice, aux);
        if (tmp) (void)hipFreeAsync(tmp, aux);
        if (e != hipSuccess) {
            // put the block back where it was (the data did not move)
            arena.release(nw);
            char *back = arena.alloc_at(old, bytes);
            (void)back;
            break;
        }
        surface_layout(sf, nw);
        moved = true;
    }
    if (moved) {
        const hipError_t es = hipStreamSynchronize(aux);
        if (e == hipSuccess) e = es;
    }
    if (e != hipSuccess && fatal == SL_OK) {
        fatal = hip_fail(e, "serving: compacting the arena");
        fatal_msg = sl_last_error(ctx);
        done_cv.notify_all();
    }
    return moved;
}

void Server::admit_locked()
{
    while (!pending.empty()) {
        HostReq &r = reqs[pending.front()];
        Surface &s = surfaces[r.surf];
        const uint64_t n_gather = (uint64_t)((s.np + kGatherChunk - 1) / kGatherChunk);
        const int64_t pieces = pieces_for(s.np);
        const uint64_t n_pair = (uint64_t)(s.np / kServeBlock * pieces);
        const uint64_t claimed = __atomic_load_n(&ctl->claimed, __ATOMIC_ACQUIRE);
        if (free_slots.empty() || tail + n_gather + n_pair - claimed > kRingCap) break;
        const size_t need = staging_bytes(s.np, r.mixed);
        char *st = arena.alloc(need);
        // first fit can leave the free bytes in pieces none of which holds the staging
        if (!st && arena.size - arena.used >= need && compact_locked()) st = arena.alloc(need);
        if (!st) break;
        const int slot = free_slots.back();
        free_slots.pop_back();
        r.slot = slot;
        r.staging = st;
        r.seq = next_seq++;
        r.n_items = n_gather + n_pair;
        r.state = ReqState::Active;
        ReqDesc d;
        d.x = s.x; d.y = s.y; d.z = s.z; d.w = s.w;
        d.x32 = s.x32; d.y32 = s.y32; d.z32 = s.z32;
        d.perm = s.perm; d.sphere = s.sphere; d.tbr = s.tbr;
        d.fx = r.fx; d.fy = r.fy; d.fz = r.fz;
        d.ux = r.ux; d.uy = r.uy; d.uz = r.uz;
        char *p = st;
        d.gx = (double *)p; p += round_up(s.np * 8, 256);
        d.gy = (double *)p; p += round_up(s.np * 8, 256);
        d.gz = (double *)p; p += round_up(s.np * 8, 256);
        if (r.mixed) {
            d.gx32 = (float *)p; p += round_up(s.np * 4, 256);
            d.gy32 = (float *)p; p += round_up(s.np * 4, 256);
            d.gz32 = (float *)p; p += round_up(s.np * 4, 256);
        } else {
            d.gx32 = d.gy32 = d.gz32 = nullptr;
        }
        d.pieces = pieces;
        d.part = nullptr;
        d.bdone = nullptr;
        if (pieces > 1) {
            d.part = (double *)p; p += round_up(pieces * 3 * s.np * 8, 256);
            d.bdone = (uint32_t *)p;
        }
        d.n = s.n;
        d.np = s.np;
        d.delta = s.delta;
        d.scale = 1.0 / (8.0 * M_PI * r.mu);
        gathers_cum[slot] += n_gather;
        items_cum[slot] += n_pair;
        d.gather_target = gathers_cum[slot];
        d.items_target = items_cum[slot];
        d.seq = r.seq;
        d.mixed = r.mixed ? 1 : 0;
        d.rho64 = r.rho64;
        memcpy((void *)&desc[slot], &d, sizeof(d));
        for (uint64_t k = 0; k < n_gather; ++k) {
            const int64_t a = (int64_t)k * kGatherChunk;
            const int64_t b = a + kGatherChunk < s.np ? a + kGatherChunk : s.np;
            ring[(tail + k) & (kRingCap - 1)] = WorkItem{(uint32_t)slot, kItemGather, (uint32_t)a, (uint32_t)b};
        }
        for (uint64_t k = 0; k < n_pair; ++k)
            ring[(tail + n_gather + k) & (kRingCap - 1)] =
                WorkItem{(uint32_t)slot, kItemPair, (uint32_t)(k / pieces), (uint32_t)(k % pieces)};
        tail += n_gather + n_pair;
        __atomic_store_n(&ctl->tail, tail, __ATOMIC_RELEASE);
        active.push_back(r.id);
        pending.pop_front();
    }
}

sl_status Server::ensure_kernel_locked()
{
    // (Re)launch only when published items may be unclaimed and no kernel is running.  The
    // claim mirror is a lower bound, so at worst this starts a kernel that idles out.
    const uint64_t claimed = __atomic_load_n(&ctl->claimed, __ATOMIC_ACQUIRE);
    if (claimed >= tail || registering > 0) return SL_OK;
    if (kernel_launched) {
        const hipError_t q = hipEventQuery(kdone);
        if (q == hipErrorNotReady) return SL_OK;          // still running
        if (q != hipSuccess) return hip_fail(q, "serving kernel");
    }
    ServeArgs a{ctl, ring, desc, ddesc, done_seq, dc,
                (uint64_t)(kIdleSeconds * clock_hz), (uint64_t)(kGatherWaitSeconds * clock_hz),
                (uint64_t)(kPollSeconds * clock_hz) + 1, stats.kernel_launches + 1};
    // All waves resident at once (so that they share one idle clock), at most kServeWavesPerSimd
    // per SIMD.
    int per_cu = 0;   // workgroups of kServeWaves waves
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void *)k_serve, kServeWaves * kWave, 0) !=
            hipSuccess ||
        per_cu < 1)
        per_cu = 1;
    const int cap = 4 * kServeWavesPerSimd / kServeWaves;
    per_cu = per_cu < cap ? per_cu : cap;
    const unsigned grid = (unsigned)(ctx->n_cu * per_cu);
    hipLaunchKernelGGL(k_serve, dim3(grid), dim3(kServeWaves * kWave), 0, kstream, a);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) e = hipEventRecord(kdone, kstream);
    if (e != hipSuccess) return hip_fail(e, "serving kernel launch");
    kernel_launched = true;
    stats.kernel_launches += 1;
    return SL_OK;
}

void Server::loop()
{
    (void)hipSetDevice(ctx->device);
    std::unique_lock<std::mutex> l(mu);
    while (!quit) {
        complete_locked();
        admit_locked();
        if (fatal == SL_OK && __atomic_load_n(&ctl->error, __ATOMIC_ACQUIRE)) {
            fatal = SL_EHIP;
            fatal_msg = "serving kernel: a work item gave up waiting for its request's density";
            done_cv.notify_all();
        }
        if (fatal == SL_OK) {
            const sl_status st = ensure_kernel_locked();
            if (st != SL_OK) {
                fatal = st;
                fatal_msg = sl_last_error(ctx);
                done_cv.notify_all();
            }
        }
        if (active.empty() && pending.empty())
            cv.wait(l);
        else
            cv.wait_for(l, std::chrono::microseconds(20));
    }
}

void server_stats(sl_ctx *ctx, sl_stats *out)
{
    Server *s = ctx->server;
    if (!s) return;
    std::lock_guard<std::mutex> l(s->mu);
    out->requests_done = s->stats.requests_done;
    out->items_done = s->stats.items_done;
    out->kernel_launches = s->stats.kernel_launches;
    out->bytes_admitted = s->arena.used;
}

}  // namespace sl

using namespace sl;

namespace {

sl_status get_server(sl_ctx *ctx, Server **out)
{
    std::lock_guard<std::mutex> l(ctx->mu);
    if (!ctx->server) {
        if (hipSetDevice(ctx->device) != hipSuccess) return fail(SL_EHIP, "serving: hipSetDevice failed");
        Server *s = new Server();
        const sl_status st = s->init(ctx);
        if (st != SL_OK) {
            s->shutdown();
            delete s;
            return st;
        }
        ctx->server = s;
    }
    *out = ctx->server;
    return SL_OK;
}

bool ranges_overlap(const void *a, const void *b, int64_t bytes)
{
    const char *x = (const char *)a, *y = (const char *)b;
    return a && b && x < y + bytes && y < x + bytes;
}

}  // namespace

extern "C" {

void sl_destroy(sl_ctx *ctx)
{
    if (!ctx) return;
    if (ctx->server) {
        (void)hipSetDevice(ctx->device);
        ctx->server->shutdown();
        delete ctx->server;
        ctx->server = nullptr;
    }
    for (auto &ev : ctx->timed)
        for (hipEvent_t e : {ev.e0, ev.e1}) (void)hipEventDestroy(e);
    for (auto ev : ctx->spare_events) (void)hipEventDestroy(ev);
    if (!ctx->splines.empty() || !ctx->fmm_ops.empty()) {
        (void)hipSetDevice(ctx->device);
        for (auto &kv : ctx->splines) (void)hipFree(kv.second);
        for (auto &kv : ctx->fmm_ops) (void)hipFree(kv.second);
    }
    if (ctx->pool) {
        // workspaces are returned stream-ordered: let the work that uses them finish first
        (void)hipSetDevice(ctx->device);
        (void)hipDeviceSynchronize();
        (void)hipMemPoolDestroy(ctx->pool);
    }
    delete ctx;
}

sl_status sl_surface_register(sl_ctx *ctx, int64_t n, const double *x, const double *y,
                              const double *z, const double *w, double delta, uint64_t *handle)
{
    if (!ctx || !handle) return fail(SL_EINVAL, "sl_surface_register: NULL argument");
    if (n < 1 || n > ((int64_t)1 << 30)) return fail(SL_EINVAL, "sl_surface_register: n must be in 1..2^30");
    if (!x || !y || !z || !w) return fail(SL_EINVAL, "sl_surface_register: NULL array");
    if (!isfinite(delta) || !(delta > 0.0)) return fail(SL_EINVAL, "sl_surface_register: bad delta");
    Server *s = nullptr;
    sl_status st = get_server(ctx, &s);
    if (st != SL_OK) return st;
    (void)hipSetDevice(ctx->device);
    const int64_t np = round_up(n, kPad);
    Surface sf;
    sf.n = n;
    sf.np = np;
    sf.delta = delta;
    {
        std::lock_guard<std::mutex> l(s->mu);
        // Requests waiting for memory go first: a surface does not overtake them.
        if (!s->pending.empty())
            return fail(SL_EBUSY, "sl_surface_register: requests are waiting for memory");
        sf.mem = s->arena.alloc(surface_bytes(np));
        if (!sf.mem)
            return fail(SL_EBUSY, "sl_surface_register: surface does not fit the HBM budget");
        // No relaunch of the persistent kernel until the surface is packed.
        s->registering += 1;
    }
    auto done_registering = [&]() {
        std::lock_guard<std::mutex> l(s->mu);
        if (--s->registering == 0) __atomic_store_n(&s->ctl->stop, 0ull, __ATOMIC_RELEASE);
        s->cv.notify_all();
    };
    surface_layout(sf, sf.mem);

    PackScratch ps;
    char *scratch = nullptr;
    hipError_t e = ws_alloc(ctx, (void **)&scratch, sort_scratch_bytes(n), s->aux);
    if (e == hipSuccess) {
        carve_sort_scratch(scratch, n, ps);
        e = launch_bbox(x, y, z, n, nullptr, nullptr, nullptr, 0, ps, s->aux);
    }
    const uint32_t *order = nullptr;
    if (e == hipSuccess) e = launch_sort_points(x, y, z, n, ps, &order, s->aux);
    if (e == hipSuccess) {
        hipLaunchKernelGGL(k_gather_surface, dim3((unsigned)(np / 256)), dim3(256), 0, s->aux, order,
                           n, x, y, z, w, ps.centre, sf.x, sf.y, sf.z, sf.w, sf.x32, sf.y32, sf.z32,
                           sf.perm, sf.sphere);
        hipLaunchKernelGGL(k_tblock_serve, dim3((unsigned)(np / kServeBlock)), dim3(kWave), 0, s->aux,
                           sf.x, sf.y, sf.z, ps.bbox, delta, sf.tbr);
        e = hipGetLastError();
    }
    if (scratch) (void)hipFreeAsync(scratch, s->aux);
    // The packing kernels run beside a busy persistent kernel where the device has room for
    // them.  If they have not finished after kRegisterWaitSeconds, ask the persistent kernel to
    // exit once its queued work is done, so that they get the device.
    if (e == hipSuccess) {
        const auto t0 = std::chrono::steady_clock::now();
        hipError_t q;
        while ((q = hipStreamQuery(s->aux)) == hipErrorNotReady &&
               std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count() < kRegisterWaitSeconds)
            std::this_thread::sleep_for(std::chrono::microseconds(50));
        if (q == hipErrorNotReady) {
            bool drain = false;
            {
                std::lock_guard<std::mutex> l(s->mu);
                if (s->kernel_launched && hipEventQuery(s->kdone) == hipErrorNotReady) {
                    __atomic_store_n(&s->ctl->stop, 1ull, __ATOMIC_RELEASE);
                    drain = true;
                }
            }
            if (drain) {
                const hipError_t ed = hipEventSynchronize(s->kdone);
                if (ed != hipSuccess) e = ed;
            }
        }
    }
    const hipError_t es = hipStreamSynchronize(s->aux);
    if (e == hipSuccess) e = es;
    done_registering();
    std::lock_guard<std::mutex> l(s->mu);
    if (e != hipSuccess) {
        s->arena.release(sf.mem);
        return hip_fail(e, "sl_surface_register");
    }
    const uint64_t h = s->next_surface++;
    s->surfaces[h] = sf;
    *handle = h;
    return SL_OK;
}

sl_status sl_surface_release(sl_ctx *ctx, uint64_t handle)
{
    if (!ctx) return fail(SL_EINVAL, "sl_surface_release: ctx is NULL");
    Server *s = ctx->server;
    if (!s) return fail(SL_ENOTFOUND, "sl_surface_release: unknown handle");
    std::lock_guard<std::mutex> l(s->mu);
    auto it = s->surfaces.find(handle);
    if (it == s->surfaces.end() || it->second.released)
        return fail(SL_ENOTFOUND, "sl_surface_release: unknown handle");
    it->second.released = true;
    if (it->second.refs == 0) s->free_surface_locked(handle);
    return SL_OK;
}

sl_status sl_request_bytes(sl_ctx *ctx, uint64_t handle, sl_precision prec, uint64_t *bytes)
{
    if (!ctx || !bytes) return fail(SL_EINVAL, "sl_request_bytes: NULL argument");
    if (prec != SL_FP64 && prec != SL_MIXED) return fail(SL_EINVAL, "sl_request_bytes: unknown precision");
    Server *s = ctx->server;
    if (!s) return fail(SL_ENOTFOUND, "sl_request_bytes: unknown surface");
    std::lock_guard<std::mutex> l(s->mu);
    auto it = s->surfaces.find(handle);
    if (it == s->surfaces.end() || it->second.released)
        return fail(SL_ENOTFOUND, "sl_request_bytes: unknown surface");
    *bytes = (uint64_t)staging_bytes(it->second.np, prec == SL_MIXED);
    return SL_OK;
}

sl_status sl_submit(sl_ctx *ctx, uint64_t handle, sl_precision prec, const double *fx,
                    const double *fy, const double *fz, double mu, double *ux, double *uy,
                    double *uz, uint64_t *request)
{
    if (!ctx || !request) return fail(SL_EINVAL, "sl_submit: NULL argument");
    if (prec != SL_FP64 && prec != SL_MIXED) return fail(SL_EINVAL, "sl_submit: unknown precision");
    if (!isfinite(mu) || !(mu > 0.0)) return fail(SL_EINVAL, "sl_submit: mu must be finite and > 0");
    if (!fx || !fy || !fz || !ux || !uy || !uz) return fail(SL_EINVAL, "sl_submit: NULL array");
    Server *s = ctx->server;
    if (!s) return fail(SL_ENOTFOUND, "sl_submit: unknown surface");
    std::lock_guard<std::mutex> l(s->mu);
    if (s->fatal != SL_OK) return fail(s->fatal, s->fatal_msg);
    auto it = s->surfaces.find(handle);
    if (it == s->surfaces.end() || it->second.released) return fail(SL_ENOTFOUND, "sl_submit: unknown surface");
    Surface &sf = it->second;
    const int64_t bytes = sf.n * 8;
    const double *ins[3] = {fx, fy, fz};
    double *outs[3] = {ux, uy, uz};
    for (int a = 0; a < 3; ++a) {
        for (int b = 0; b < 3; ++b)
            if (ranges_overlap(outs[a], ins[b], bytes)) return fail(SL_EINVAL, "sl_submit: output aliases input");
        for (int b = a + 1; b < 3; ++b)
            if (ranges_overlap(outs[a], outs[b], bytes)) return fail(SL_EINVAL, "sl_submit: outputs overlap");
    }
    if (staging_bytes(sf.np, prec == SL_MIXED) > s->arena.size)
        return fail(SL_EBUSY, "sl_submit: request staging exceeds the whole HBM budget");
    if ((uint64_t)((sf.np + kGatherChunk - 1) / kGatherChunk + sf.np / kServeBlock) > kRingCap)
        return fail(SL_EINVAL, "sl_submit: surface needs more work items than the queue holds");
    HostReq r;
    r.id = s->next_req++;
    r.surf = handle;
    r.mixed = prec == SL_MIXED;
    r.fx = fx; r.fy = fy; r.fz = fz;
    r.ux = ux; r.uy = uy; r.uz = uz;
    r.mu = mu;
    r.rho64 = ctx->rho64;
    sf.refs += 1;
    s->reqs[r.id] = r;
    s->pending.push_back(r.id);
    // Admit now when the memory is there, so that the request holds its staging from this call
    // on (a later registration cannot take it).
    s->admit_locked();
    *request = r.id;
    s->cv.notify_all();
    return SL_OK;
}

sl_status sl_poll(sl_ctx *ctx, uint64_t request, int *done)
{
    if (!ctx || !done) return fail(SL_EINVAL, "sl_poll: NULL argument");
    Server *s = ctx->server;
    if (!s) return fail(SL_ENOTFOUND, "sl_poll: unknown request");
    std::lock_guard<std::mutex> l(s->mu);
    auto it = s->reqs.find(request);
    if (it == s->reqs.end()) return fail(SL_ENOTFOUND, "sl_poll: unknown request");
    if (s->fatal != SL_OK) return fail(s->fatal, s->fatal_msg);
    *done = it->second.state == ReqState::Done;
    if (*done) s->reqs.erase(it);
    return SL_OK;
}

sl_status sl_wait(sl_ctx *ctx, uint64_t request, double timeout_s)
{
    if (!ctx) return fail(SL_EINVAL, "sl_wait: ctx is NULL");
    if (!(timeout_s >= 0.0)) return fail(SL_EINVAL, "sl_wait: negative timeout");
    Server *s = ctx->server;
    if (!s) return fail(SL_ENOTFOUND, "sl_wait: unknown request");
    std::unique_lock<std::mutex> l(s->mu);
    auto it = s->reqs.find(request);
    if (it == s->reqs.end()) return fail(SL_ENOTFOUND, "sl_wait: unknown request");
    const auto deadline = std::chrono::steady_clock::now() +
                          std::chrono::microseconds((int64_t)(timeout_s * 1e6));
    while (s->reqs[request].state != ReqState::Done && s->fatal == SL_OK) {
        if (s->done_cv.wait_until(l, deadline) == std::cv_status::timeout &&
            s->reqs[request].state != ReqState::Done)
            return fail(SL_ETIMEDOUT, "sl_wait: timed out");
    }
    if (s->fatal != SL_OK) return fail(s->fatal, s->fatal_msg);
    s->reqs.erase(request);
    return SL_OK;
}

}  // extern "C"
