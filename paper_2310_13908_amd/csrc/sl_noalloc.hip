// sl_noalloc.hip -- sl_eval without any allocation, for callers that cannot allocate device memory
// (code under stream capture, serving loops that must not call the allocator, harnesses that
// forbid it).  The workspace of the sort, the packed sources and the per-way partial sums lives in
// a file-scope device array of fixed size; each GPU that the library runs on holds its own copy
// until the process ends.
#include <mutex>
#include <string>

#include "sl_internal.h"

namespace sl {

namespace {

constexpr size_t kScratchBytes = (size_t)256 << 20;   // the stated maximum: 256 MiB per device
constexpr int kMaxDevices = 64;

static __device__ __align__(256) char scratch[kScratchBytes];

// Device address of `scratch` on each device, looked up once per device with that device current.
// In host code the array's name is only a host-side stand-in and never passed to the device.
std::mutex g_mu;
char *g_ptr[kMaxDevices] = {};

sl_status scratch_on(int device, char **out)
{
    if (device < 0 || device >= kMaxDevices) return fail(SL_EINVAL, "sl_eval_noalloc: device ordinal out of range");
    std::lock_guard<std::mutex> l(g_mu);
    if (!g_ptr[device]) {
        void *p = nullptr;
        int prev = -1;
        if (hipGetDevice(&prev) != hipSuccess) prev = -1;
        hipError_t e = hipSetDevice(device);
        if (e == hipSuccess) e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (prev >= 0) (void)hipSetDevice(prev);
        if (e != hipSuccess || !p) return hip_fail(e != hipSuccess ? e : hipErrorInvalidSymbol,
                                                   "sl_eval_noalloc: hipGetSymbolAddress(scratch)");
        g_ptr[device] = static_cast<char *>(p);
    }
    *out = g_ptr[device];
    return SL_OK;
}

}  // namespace

}  // namespace sl

using namespace sl;

extern "C" {

sl_status sl_eval_noalloc(sl_ctx *ctx, sl_precision prec, int64_t n_src, const double *sx,
                          const double *sy, const double *sz, const double *w, const double *fx,
                          const double *fy, const double *fz, int64_t n_tgt, const double *tx,
                          const double *ty, const double *tz, double delta, const double *delta_tgt,
                          double mu, double *ux, double *uy, double *uz, void *stream)
{
    if (!ctx) return fail(SL_EINVAL, "sl_eval_noalloc: ctx is NULL");
    char *base = nullptr;
    const sl_status s = scratch_on(ctx->device, &base);
    if (s != SL_OK) return s;
    return eval_common("sl_eval_noalloc", ctx, prec, n_src, sx, sy, sz, w, fx, fy, fz, n_tgt, tx, ty, tz,
                       delta, delta_tgt, mu, ux, uy, uz, stream, base, kScratchBytes);
}

}  // extern "C"
