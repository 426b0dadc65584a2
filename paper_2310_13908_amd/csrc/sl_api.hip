// sl_api.hip -- C ABI entry points: context, parameters, one-shot evaluation.
#include <math.h>
#include <string.h>

#include <algorithm>

#include "sl_internal.h"

namespace sl {

namespace {
thread_local std::string g_last_error;

// Makes the context's device current for the duration of a call and restores the caller's.
struct DeviceGuard {
    int prev = -1;
    bool ok = false;
    explicit DeviceGuard(int dev)
    {
        if (hipGetDevice(&prev) != hipSuccess) prev = -1;
        ok = hipSetDevice(dev) == hipSuccess;
    }
    ~DeviceGuard()
    {
        if (prev >= 0) (void)hipSetDevice(prev);
    }
};

struct Range {
    const void *p;
    int64_t bytes;
};

bool overlaps(const Range &a, const Range &b)
{
    if (!a.p || !b.p || a.bytes <= 0 || b.bytes <= 0) return false;
    const char *a0 = (const char *)a.p, *b0 = (const char *)b.p;
    return a0 < b0 + b.bytes && b0 < a0 + a.bytes;
}

bool finite_pos(double v) { return isfinite(v) && v > 0.0; }

constexpr int64_t kMaxPoints = (int64_t)1 << 30;

}  // namespace

sl_status fail(sl_status s, const std::string &msg)
{
    g_last_error = msg;
    return s;
}

sl_status hip_fail(hipError_t e, const char *what)
{
    return fail(e == hipErrorOutOfMemory ? SL_ENOMEM : SL_EHIP,
                std::string(what) + ": " + hipGetErrorString(e));
}

// Workspace of one sl_eval call, carved from a single stream-ordered allocation.
struct EvalWorkspace {
    PackScratch ps;
    SrcOut so;
    TgtOut to;
    double *part;
    void *tblock;
};

static size_t carve(char *base, EvalWorkspace &w, int64_t n_sort, int64_t np_s, int64_t np_t,
                    bool distinct, bool mixed, bool vard, int n_ways)
{
    size_t off = 0;
    auto take = [&](size_t bytes) -> char * {
        char *p = base ? base + off : nullptr;
        off += (size_t)round_up((int64_t)bytes, 256);
        return p;
    };
    char *sort_base = take(sort_scratch_bytes(n_sort));
    if (base) carve_sort_scratch(sort_base, n_sort, w.ps);
    memset(&w.so, 0, sizeof(w.so));
    memset(&w.to, 0, sizeof(w.to));
    w.so.d = (double *)take(np_s * 64);
    if (mixed) w.so.f32 = (float *)take(np_s * 32);
    w.so.sphere = (double4 *)take(np_s / kCluster * sizeof(double4));
    if (!distinct) {   // targets = sources: structure-of-arrays positions for the target side
        w.so.x = (double *)take(np_s * 8); w.so.y = (double *)take(np_s * 8); w.so.z = (double *)take(np_s * 8);
        if (mixed) {
            w.so.x32 = (float *)take(np_s * 4); w.so.y32 = (float *)take(np_s * 4); w.so.z32 = (float *)take(np_s * 4);
        }
        w.so.perm = (int32_t *)take(np_s * 4);
    }
    if (distinct) {
        w.to.x = (double *)take(np_t * 8); w.to.y = (double *)take(np_t * 8); w.to.z = (double *)take(np_t * 8);
        if (mixed) {
            w.to.x32 = (float *)take(np_t * 4); w.to.y32 = (float *)take(np_t * 4); w.to.z32 = (float *)take(np_t * 4);
        }
        w.to.perm = (int32_t *)take(np_t * 4);
    }
    if (vard) w.to.delta = (double *)take(np_t * 8);
    w.part = (double *)take((size_t)n_ways * 3 * np_t * 8);
    w.tblock = take(tblock_scratch_bytes((int)(np_t / kWave)));   // enough for any R >= 1
    return off;
}

// Largest padded target count for which the FP64 pair kernel keeps one target a lane by default.
constexpr int64_t kFp64OneTargetMaxN = 1 << 17;

// Validation and launch sequence of sl_eval and sl_eval_noalloc.  fixed == nullptr: the workspace
// is allocated and freed stream-ordered; otherwise the fixed_bytes at `fixed` are used.
sl_status eval_common(const char *who, sl_ctx *ctx, sl_precision prec, int64_t n_src, const double *sx,
                      const double *sy, const double *sz, const double *w, const double *fx,
                      const double *fy, const double *fz, int64_t n_tgt, const double *tx,
                      const double *ty, const double *tz, double delta, const double *delta_tgt,
                      double mu, double *ux, double *uy, double *uz, void *stream, char *fixed,
                      size_t fixed_bytes)
{
    const std::string w_ = std::string(who) + ": ";
    g_last_error.clear();
    if (!ctx) return fail(SL_EINVAL, w_ + "ctx is NULL");
    if (prec != SL_FP64 && prec != SL_MIXED) return fail(SL_EINVAL, w_ + "unknown precision");
    if (n_src < 0 || n_tgt < 0) return fail(SL_EINVAL, w_ + "negative size");
    if (n_src > kMaxPoints || n_tgt > kMaxPoints) return fail(SL_EINVAL, w_ + "more than 2^30 points");
    if (!finite_pos(mu)) return fail(SL_EINVAL, w_ + "mu must be finite and > 0");
    if (!delta_tgt && !finite_pos(delta)) return fail(SL_EINVAL, w_ + "delta must be finite and > 0");
    const bool same = !tx && !ty && !tz;
    if (!same && (!tx || !ty || !tz)) return fail(SL_EINVAL, w_ + "tx, ty, tz must be all NULL or all set");
    if (same && n_tgt != n_src) return fail(SL_EINVAL, w_ + "targets = sources needs n_tgt == n_src");
    if (n_tgt > 0 && (!ux || !uy || !uz)) return fail(SL_EINVAL, w_ + "output pointer is NULL");
    if (n_src > 0 && (!sx || !sy || !sz || !w || !fx || !fy || !fz))
        return fail(SL_EINVAL, w_ + "source pointer is NULL");
    {
        const Range outs[3] = {{ux, n_tgt * 8}, {uy, n_tgt * 8}, {uz, n_tgt * 8}};
        const Range ins[11] = {{sx, n_src * 8}, {sy, n_src * 8}, {sz, n_src * 8}, {w, n_src * 8},
                               {fx, n_src * 8}, {fy, n_src * 8}, {fz, n_src * 8}, {tx, n_tgt * 8},
                               {ty, n_tgt * 8}, {tz, n_tgt * 8}, {delta_tgt, n_tgt * 8}};
        for (int a = 0; a < 3; ++a) {
            for (int b = a + 1; b < 3; ++b)
                if (overlaps(outs[a], outs[b])) return fail(SL_EINVAL, w_ + "outputs overlap");
            for (const Range &r : ins)
                if (overlaps(outs[a], r)) return fail(SL_EINVAL, w_ + "output aliases an input");
        }
    }
    if (n_tgt == 0) return SL_OK;

    DeviceGuard g(ctx->device);
    if (!g.ok) return fail(SL_EHIP, w_ + "hipSetDevice failed");
    hipStream_t st = (hipStream_t)stream;
    if (n_src == 0) {
        SL_HIP(launch_fill_zero(ux, uy, uz, n_tgt, st));
        return SL_OK;
    }

    const bool mixed = prec == SL_MIXED;
    const bool vard = delta_tgt != nullptr;
    const int64_t np_s = round_up(n_src, kPad);
    const int64_t np_t = same ? np_s : round_up(n_tgt, kPad);
    const int64_t n_sort = std::max(n_src, same ? (int64_t)0 : n_tgt);
    int R, wps;
    {
        std::lock_guard<std::mutex> l(ctx->mu);
        R = ctx->targets_per_lane;
        wps = ctx->waves_per_simd;
    }
    // Measured on MI355X: the single-precision loops want occupancy; FP64 wants occupancy while
    // its near field (longer loops, more registers at two targets a lane) weighs in, and two
    // targets a lane once the far field dominates (N = 24,576: 0.98 against 1.07 ms; N = 393,216:
    // 125.5 against 119.6 ms).
    if (R == 0) R = mixed ? 1 : (np_t <= kFp64OneTargetMaxN ? 1 : 2);
    PairPlan plan = plan_pairs(np_s, np_t, R, ctx->n_cu * 4 * wps, mixed);
    plan.n_cu = ctx->n_cu;

    EvalWorkspace ws;
    size_t bytes = carve(nullptr, ws, n_sort, np_s, np_t, !same, mixed, vard, plan.n_ways);
    char *base = fixed;
    if (fixed) {
        // a caller-sized region: fewer ways (larger work items) until the partial sums fit
        const size_t per_way = (size_t)round_up(3 * np_t * 8, 256);
        if (bytes > fixed_bytes) {
            const size_t rest = bytes - (size_t)plan.n_ways * per_way;
            const int64_t k_fit = rest < fixed_bytes ? (int64_t)((fixed_bytes - rest) / per_way) : 0;
            if (k_fit < 1)
                return fail(SL_EINVAL, w_ + "the workspace for " + std::to_string(n_src) + " sources and " +
                                           std::to_string(n_tgt) + " targets (" + std::to_string(rest + per_way) +
                                           " bytes) exceeds the " + std::to_string(fixed_bytes) + "-byte scratch");
            plan.n_ways = (int)k_fit;
            bytes = carve(nullptr, ws, n_sort, np_s, np_t, !same, mixed, vard, plan.n_ways);
        }
    } else {
        hipError_t ea = ws_alloc(ctx, (void **)&base, bytes, st);
        if (ea != hipSuccess) return hip_fail(ea, (w_ + "workspace").c_str());
    }
    carve(base, ws, n_sort, np_s, np_t, !same, mixed, vard, plan.n_ways);

    double rho64;
    {
        std::lock_guard<std::mutex> l(ctx->mu);
        rho64 = ctx->rho64;
    }
    // far clusters: s = 1 to the working precision, and (mixed) outside the FP64 zone
    const double far_cut = mixed ? std::max(kRhoExact32, rho64) : kRhoExact64;
    // targets = sources with one delta: the source gather also writes the target records
    TRecOut trec = {};
    const int G = pair_group_size(mixed);
    if (same && !vard && plan.R * G <= 4) {
        trec.rec = reinterpret_cast<TBlockRec *>(ws.tblock);
        trec.ctr = pair_counter(ws.tblock, plan.n_tblocks);
        trec.bbox = ws.ps.bbox;
        trec.gap_far = far_cut * delta;
        trec.R = plan.R;
        trec.G = G;
        trec.n_tblocks = plan.n_tblocks;
        trec.mixed = mixed ? 1 : 0;
    }

    hipError_t e = launch_bbox(sx, sy, sz, n_src, tx, ty, tz, same ? 0 : n_tgt, ws.ps, st);
    const uint32_t *order = nullptr;
    if (e == hipSuccess) e = launch_sort_points(sx, sy, sz, n_src, ws.ps, &order, st);
    if (e == hipSuccess)
        e = launch_gather_src(order, n_src, np_s, sx, sy, sz, w, fx, fy, fz, ws.ps.centre, ws.so, trec, st);
    TgtView tv;
    if (same) {
        tv.x = ws.so.x; tv.y = ws.so.y; tv.z = ws.so.z;
        tv.x32 = ws.so.x32; tv.y32 = ws.so.y32; tv.z32 = ws.so.z32;
        tv.perm = ws.so.perm;
        if (vard && e == hipSuccess) {
            TgtOut d = {};
            d.delta = ws.to.delta;
            e = launch_gather_tgt(order, n_tgt, np_t, nullptr, nullptr, nullptr, delta_tgt,
                                  ws.ps.centre, d, st);
        }
    } else {
        if (e == hipSuccess) e = launch_sort_points(tx, ty, tz, n_tgt, ws.ps, &order, st);
        if (e == hipSuccess)
            e = launch_gather_tgt(order, n_tgt, np_t, tx, ty, tz, delta_tgt, ws.ps.centre, ws.to, st);
        tv.x = ws.to.x; tv.y = ws.to.y; tv.z = ws.to.z;
        tv.x32 = ws.to.x32; tv.y32 = ws.to.y32; tv.z32 = ws.to.z32;
        tv.perm = ws.to.perm;
    }
    tv.delta = vard ? ws.to.delta : nullptr;
    tv.np = np_t;
    tv.n = n_tgt;

    PairArgs pa;
    pa.s = SrcView{ws.so.d, ws.so.f32, ws.so.sphere, np_s};
    pa.t = tv;
    pa.delta = vard ? 1.0 : delta;
    pa.rho64 = rho64;
    pa.far_cut = far_cut;
    pa.records_ready = trec.rec ? 1 : 0;
    pa.n_tblocks = plan.n_tblocks;
    pa.n_ways = plan.n_ways;
    pa.part = ws.part;
    pa.bbox = ws.ps.bbox;
    pa.tblock_scratch = ws.tblock;
    PairTiming tev{nullptr, nullptr};
    if (ctx->timing && !fixed && e == hipSuccess) {
        std::lock_guard<std::mutex> l(ctx->mu);
        for (hipEvent_t *ev : {&tev.e0, &tev.e1}) {
            if (!ctx->spare_events.empty()) {
                *ev = ctx->spare_events.back();
                ctx->spare_events.pop_back();
            } else if (e == hipSuccess) {
                e = hipEventCreate(ev);
            }
        }
    }
    if (e == hipSuccess) e = launch_pair(pa, plan, mixed, vard, st, tev.e1 ? &tev : nullptr);
    if (tev.e1 && e == hipSuccess) {
        std::lock_guard<std::mutex> l(ctx->mu);
        ctx->timed.push_back(tev);
    }
    if (e == hipSuccess)
        e = launch_reduce(ws.part, plan.n_ways, np_t, tv.perm, 1.0 / (8.0 * M_PI * mu), ux, uy, uz, st);
    const hipError_t ef = fixed ? hipSuccess : hipFreeAsync(base, st);
    if (e != hipSuccess) return hip_fail(e, (w_ + "kernel launch").c_str());
    if (ef != hipSuccess) return hip_fail(ef, (w_ + "hipFreeAsync").c_str());
    return SL_OK;
}


}  // namespace sl

using namespace sl;

extern "C" {

const char *sl_last_error(const sl_ctx *ctx)
{
    (void)ctx;   // the message is kept per thread, whatever the context
    return g_last_error.c_str();
}

sl_status sl_create(int device, size_t hbm_budget_bytes, sl_ctx **out)
{
    g_last_error.clear();
    if (!out) return fail(SL_EINVAL, "sl_create: out is NULL");
    *out = nullptr;
    int n = 0;
    if (hipGetDeviceCount(&n) != hipSuccess || device < 0 || device >= n)
        return fail(SL_EINVAL, "sl_create: no such HIP device");
    DeviceGuard g(device);
    if (!g.ok) return fail(SL_EHIP, "sl_create: hipSetDevice failed");
    hipDeviceProp_t prop;
    SL_HIP(hipGetDeviceProperties(&prop, device));
    if (strncmp(prop.gcnArchName, "gfx950", 6) != 0)
        return fail(SL_EINVAL, std::string("sl_create: built for gfx950, device is ") + prop.gcnArchName);
    size_t free_b = 0, total_b = 0;
    SL_HIP(hipMemGetInfo(&free_b, &total_b));
    hipMemPoolProps props;
    memset(&props, 0, sizeof(props));
    props.allocType = hipMemAllocationTypePinned;
    props.handleTypes = hipMemHandleTypeNone;
    props.location.type = hipMemLocationTypeDevice;
    props.location.id = device;
    hipMemPool_t pool = nullptr;
    SL_HIP(hipMemPoolCreate(&pool, &props));
    uint64_t keep = UINT64_MAX;
    const hipError_t ep = hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &keep);
    if (ep != hipSuccess) {
        (void)hipMemPoolDestroy(pool);
        return hip_fail(ep, "sl_create: hipMemPoolSetAttribute");
    }
    sl_ctx *c = new sl_ctx();
    c->pool = pool;
    c->device = device;
    c->n_cu = prop.multiProcessorCount;
    c->budget = hbm_budget_bytes ? hbm_budget_bytes : (size_t)(0.9 * (double)free_b);
    *out = c;
    return SL_OK;
}

sl_status sl_set_param(sl_ctx *ctx, sl_param key, double value)
{
    if (!ctx) return fail(SL_EINVAL, "sl_set_param: ctx is NULL");
    if (key == SL_PARAM_RHO64) {
        if (!isfinite(value) || value < kRho64Min)
            return fail(SL_EINVAL, "sl_set_param: rho64 must be finite and >= 0");
        std::lock_guard<std::mutex> l(ctx->mu);
        ctx->rho64 = value;
        return SL_OK;
    }
    if (key == SL_PARAM_TARGETS_PER_LANE) {
        if (value != 0.0 && value != 1.0 && value != 2.0 && value != 4.0)
            return fail(SL_EINVAL, "sl_set_param: targets per lane is 0 (automatic), 1, 2 or 4");
        std::lock_guard<std::mutex> l(ctx->mu);
        ctx->targets_per_lane = (int)value;
        return SL_OK;
    }
    if (key == SL_PARAM_WAVES_PER_SIMD) {
        if (!(value >= 1.0 && value <= 256.0) || value != (double)(int)value)
            return fail(SL_EINVAL, "sl_set_param: waves per SIMD is an integer in 1..256");
        std::lock_guard<std::mutex> l(ctx->mu);
        ctx->waves_per_simd = (int)value;
        return SL_OK;
    }
    if (key == SL_PARAM_KERNEL_TIMING) {
        if (value != 0.0 && value != 1.0) return fail(SL_EINVAL, "sl_set_param: timing is 0 or 1");
        std::lock_guard<std::mutex> l(ctx->mu);
        ctx->timing = value == 1.0;
        return SL_OK;
    }
    return fail(SL_EINVAL, "sl_set_param: unknown key");
}

sl_status sl_get_param(const sl_ctx *ctx, sl_param key, double *value)
{
    if (!ctx || !value) return fail(SL_EINVAL, "sl_get_param: NULL argument");
    if (key == SL_PARAM_RHO64) {
        *value = ctx->rho64;
        return SL_OK;
    }
    if (key == SL_PARAM_KERNEL_TIMING) {
        *value = ctx->timing ? 1.0 : 0.0;
        return SL_OK;
    }
    if (key == SL_PARAM_TARGETS_PER_LANE) {
        *value = ctx->targets_per_lane;
        return SL_OK;
    }
    if (key == SL_PARAM_WAVES_PER_SIMD) {
        *value = ctx->waves_per_simd;
        return SL_OK;
    }
    return fail(SL_EINVAL, "sl_get_param: unknown key");
}

sl_status sl_get_stats(sl_ctx *ctx, sl_stats *out)
{
    if (!ctx || !out) return fail(SL_EINVAL, "sl_get_stats: NULL argument");
    memset(out, 0, sizeof(*out));
    {
        std::lock_guard<std::mutex> l(ctx->mu);
        DeviceGuard g(ctx->device);
        for (auto &ev : ctx->timed) {
            float ms = 0.0f;
            SL_HIP(hipEventSynchronize(ev.e1));
            SL_HIP(hipEventElapsedTime(&ms, ev.e0, ev.e1));
            ctx->pair_ms += ms;
            ctx->pair_launches += 1;
            for (hipEvent_t e : {ev.e0, ev.e1}) ctx->spare_events.push_back(e);
        }
        ctx->timed.clear();
        out->pair_launches = ctx->pair_launches;
        out->pair_ms = ctx->pair_ms;
    }
    server_stats(ctx, out);
    return SL_OK;
}

sl_status sl_patch_delta(sl_ctx *ctx, int64_t n_patches, int64_t n, const double *x, const double *y,
                         const double *z, double C, double *delta_out, void *stream)
{
    g_last_error.clear();
    if (!ctx) return fail(SL_EINVAL, "sl_patch_delta: ctx is NULL");
    if (n_patches < 1 || n < 2)
        return fail(SL_EINVAL, "sl_patch_delta: need n_patches >= 1 and n >= 2 (a one-node patch has no neighbours)");
    if (n > 32768 || n_patches > kMaxPoints / (n * n))
        return fail(SL_EINVAL, "sl_patch_delta: more than 2^30 points");
    if (!finite_pos(C)) return fail(SL_EINVAL, "sl_patch_delta: C must be finite and > 0");
    if (!x || !y || !z || !delta_out) return fail(SL_EINVAL, "sl_patch_delta: NULL array");
    const int64_t bytes = n_patches * n * n * 8;
    const Range out{delta_out, bytes};
    for (const void *in : {(const void *)x, (const void *)y, (const void *)z})
        if (overlaps(out, Range{in, bytes}))
            return fail(SL_EINVAL, "sl_patch_delta: delta_out aliases an input");
    DeviceGuard g(ctx->device);
    if (!g.ok) return fail(SL_EHIP, "sl_patch_delta: hipSetDevice failed");
    const hipError_t e = launch_patch_delta(n_patches, n, x, y, z, C, delta_out, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "sl_patch_delta: kernel launch");
    return SL_OK;
}

sl_status sl_eval(sl_ctx *ctx, sl_precision prec, int64_t n_src, const double *sx,
                  const double *sy, const double *sz, const double *w, const double *fx,
                  const double *fy, const double *fz, int64_t n_tgt, const double *tx,
                  const double *ty, const double *tz, double delta, const double *delta_tgt,
                  double mu, double *ux, double *uy, double *uz, void *stream)
{
    return eval_common("sl_eval", ctx, prec, n_src, sx, sy, sz, w, fx, fy, fz, n_tgt, tx, ty, tz, delta,
                       delta_tgt, mu, ux, uy, uz, stream, nullptr, 0);
}

}  // extern "C"
