"""ctypes binding of libstokeslet.so: the C ABI of include/stokeslet.h under the same names.

Argument marshalling only -- every step of the computation runs in the library's HIP
kernels.  Loading fails loudly when the library has not been built; there is no fallback.
"""
from __future__ import annotations

import ctypes
import os

_PKG = os.path.dirname(os.path.abspath(__file__))
# SL_LIB may name another build of the same library (the host-sanitized one, for its tests).
LIB_PATH = os.environ.get("SL_LIB") or os.path.join(_PKG, "libstokeslet.so")

SL_OK, SL_EINVAL, SL_ENOMEM, SL_EBUSY, SL_EHIP, SL_ENOTFOUND, SL_ETIMEDOUT = 0, -1, -2, -3, -4, -5, -6
SL_FP64, SL_MIXED = 0, 1
SL_PARAM_RHO64 = 0
SL_PARAM_KERNEL_TIMING = 1
SL_PARAM_TARGETS_PER_LANE = 2
SL_PARAM_WAVES_PER_SIMD = 3

STATUS_NAMES = {0: "SL_OK", -1: "SL_EINVAL", -2: "SL_ENOMEM", -3: "SL_EBUSY", -4: "SL_EHIP",
                -5: "SL_ENOTFOUND", -6: "SL_ETIMEDOUT"}

# Every symbol include/stokeslet.h declares.
EXPORTED = ["sl_create", "sl_destroy", "sl_last_error", "sl_set_param", "sl_get_param", "sl_eval",
            "sl_eval_noalloc", "sl_eval_fmm", "sl_patch_delta", "sl_eval_upsampled",
            "sl_surface_register", "sl_surface_release", "sl_submit", "sl_poll", "sl_wait",
            "sl_request_bytes", "sl_get_stats"]


class SlError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


class sl_stats(ctypes.Structure):
    _fields_ = [("requests_done", ctypes.c_uint64), ("items_done", ctypes.c_uint64),
                ("kernel_launches", ctypes.c_uint64), ("bytes_admitted", ctypes.c_uint64),
                ("pair_launches", ctypes.c_uint64), ("pair_ms", ctypes.c_double)]


_lib = None


def load():
    """Load the built library (no build, no fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it first "
                          "(python -m paper_2310_13908_amd.build)")
    # torch provides the device memory and streams the library works on; load its HIP runtime
    # first so that the library binds to the same runtime instance (one libamdhip64 per process).
    import torch  # noqa: F401
    lib = ctypes.CDLL(LIB_PATH)
    P, V = ctypes.c_void_p, ctypes.c_void_p
    i64, u64, d, i32 = ctypes.c_int64, ctypes.c_uint64, ctypes.c_double, ctypes.c_int
    sig = {
        "sl_create": ([i32, ctypes.c_size_t, ctypes.POINTER(P)], i32),
        "sl_destroy": ([P], None),
        "sl_last_error": ([P], ctypes.c_char_p),
        "sl_set_param": ([P, i32, d], i32),
        "sl_get_param": ([P, i32, ctypes.POINTER(d)], i32),
        "sl_eval": ([P, i32, i64, V, V, V, V, V, V, V, i64, V, V, V, d, V, d, V, V, V, V], i32),
        "sl_eval_noalloc": ([P, i32, i64, V, V, V, V, V, V, V, i64, V, V, V, d, V, d, V, V, V, V], i32),
        "sl_eval_fmm": ([P, i32, i64, V, V, V, V, V, V, V, d, V, d, i32, i32, i32, V, V, V, V, V], i32),
        "sl_patch_delta": ([P, i64, i64, V, V, V, d, V, V], i32),
        "sl_eval_upsampled": ([P, i32, i64, i64, i32, V, V, V, V, V, V, V, V, d, d, V, V, V, V], i32),
        "sl_surface_register": ([P, i64, V, V, V, V, d, ctypes.POINTER(u64)], i32),
        "sl_surface_release": ([P, u64], i32),
        "sl_submit": ([P, u64, i32, V, V, V, d, V, V, V, ctypes.POINTER(u64)], i32),
        "sl_poll": ([P, u64, ctypes.POINTER(i32)], i32),
        "sl_wait": ([P, u64, d], i32),
        "sl_request_bytes": ([P, u64, i32, ctypes.POINTER(u64)], i32),
        "sl_get_stats": ([P, ctypes.POINTER(sl_stats)], i32),
    }
    for name, (args, res) in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = res
    _lib = lib
    return lib


def check(status: int, what: str = ""):
    if status != SL_OK:
        msg = load().sl_last_error(None).decode(errors="replace")
        raise SlError(status, f"{what}: {msg}" if what else msg)
    return status


# ------------------------------------------------------------------------------------------
# Same-name wrappers (pointers are Python ints: device addresses / stream handles).
# ------------------------------------------------------------------------------------------
def sl_create(device: int = 0, hbm_budget_bytes: int = 0):
    ctx = ctypes.c_void_p()
    check(load().sl_create(device, hbm_budget_bytes, ctypes.byref(ctx)), "sl_create")
    return ctx


def sl_destroy(ctx) -> None:
    load().sl_destroy(ctx)


def sl_last_error(ctx=None) -> str:
    return load().sl_last_error(ctx).decode(errors="replace")


def sl_set_param(ctx, key: int, value: float) -> int:
    return load().sl_set_param(ctx, key, value)


def sl_get_param(ctx, key: int) -> float:
    v = ctypes.c_double()
    check(load().sl_get_param(ctx, key, ctypes.byref(v)), "sl_get_param")
    return v.value


def sl_eval(ctx, prec, n_src, sx, sy, sz, w, fx, fy, fz, n_tgt, tx, ty, tz, delta, delta_tgt,
            mu, ux, uy, uz, stream) -> int:
    return load().sl_eval(ctx, prec, n_src, sx, sy, sz, w, fx, fy, fz, n_tgt, tx, ty, tz, delta,
                          delta_tgt, mu, ux, uy, uz, stream)


def sl_eval_noalloc(ctx, prec, n_src, sx, sy, sz, w, fx, fy, fz, n_tgt, tx, ty, tz, delta,
                    delta_tgt, mu, ux, uy, uz, stream) -> int:
    return load().sl_eval_noalloc(ctx, prec, n_src, sx, sy, sz, w, fx, fy, fz, n_tgt, tx, ty, tz,
                                  delta, delta_tgt, mu, ux, uy, uz, stream)


def sl_eval_fmm(ctx, prec, n, x, y, z, w, fx, fy, fz, delta, delta_tgt, mu, k, p_edge, max_iter,
                ux, uy, uz, labels_out, stream) -> int:
    return load().sl_eval_fmm(ctx, prec, n, x, y, z, w, fx, fy, fz, delta, delta_tgt, mu, k, p_edge,
                              max_iter, ux, uy, uz, labels_out, stream)


def sl_patch_delta(ctx, n_patches, n, x, y, z, C, delta_out, stream) -> int:
    return load().sl_patch_delta(ctx, n_patches, n, x, y, z, C, delta_out, stream)


def sl_eval_upsampled(ctx, prec, n_patches, n, factor, x, y, z, W, psi_up, fx, fy, fz, C, mu, ux,
                      uy, uz, stream) -> int:
    return load().sl_eval_upsampled(ctx, prec, n_patches, n, factor, x, y, z, W, psi_up, fx, fy, fz,
                                    C, mu, ux, uy, uz, stream)


def sl_surface_register(ctx, n, x, y, z, w, delta):
    h = ctypes.c_uint64()
    st = load().sl_surface_register(ctx, n, x, y, z, w, delta, ctypes.byref(h))
    return st, h.value


def sl_surface_release(ctx, handle) -> int:
    return load().sl_surface_release(ctx, handle)


def sl_submit(ctx, handle, prec, fx, fy, fz, mu, ux, uy, uz):
    r = ctypes.c_uint64()
    st = load().sl_submit(ctx, handle, prec, fx, fy, fz, mu, ux, uy, uz, ctypes.byref(r))
    return st, r.value


def sl_poll(ctx, request):
    done = ctypes.c_int()
    st = load().sl_poll(ctx, request, ctypes.byref(done))
    return st, bool(done.value)


def sl_wait(ctx, request, timeout_s: float) -> int:
    return load().sl_wait(ctx, request, timeout_s)


def sl_request_bytes(ctx, handle, prec):
    b = ctypes.c_uint64()
    st = load().sl_request_bytes(ctx, handle, prec, ctypes.byref(b))
    return st, b.value


def sl_get_stats(ctx) -> sl_stats:
    s = sl_stats()
    check(load().sl_get_stats(ctx, ctypes.byref(s)), "sl_get_stats")
    return s
