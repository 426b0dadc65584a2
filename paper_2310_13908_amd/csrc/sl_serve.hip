// sl_serve.hip -- resident surfaces and the continuously batched persistent kernel.
#include "sl_internal.h"

using namespace sl;

void sl::server_stats(sl_ctx *, sl_stats *) {}

extern "C" {

void sl_destroy(sl_ctx *ctx)
{
    if (!ctx) return;
    for (auto &ev : ctx->timed)
        for (hipEvent_t e : {ev.e0, ev.e1, ev.e2}) (void)hipEventDestroy(e);
    for (auto ev : ctx->spare_events) (void)hipEventDestroy(ev);
    delete ctx;
}

sl_status sl_surface_register(sl_ctx *, int64_t, const double *, const double *, const double *,
                              const double *, double, uint64_t *)
{
    return fail(SL_EINVAL, "serving not built");
}
sl_status sl_surface_release(sl_ctx *, uint64_t) { return fail(SL_EINVAL, "serving not built"); }
sl_status sl_submit(sl_ctx *, uint64_t, sl_precision, const double *, const double *,
                    const double *, double, double *, double *, double *, uint64_t *)
{
    return fail(SL_EINVAL, "serving not built");
}
sl_status sl_poll(sl_ctx *, uint64_t, int *) { return fail(SL_EINVAL, "serving not built"); }
sl_status sl_wait(sl_ctx *, uint64_t, double) { return fail(SL_EINVAL, "serving not built"); }
}
