"""MI355X (gfx950) regularized Stokes single layer (Agarwal & Biros, Sec. 3.4).

The computation lives in ``libstokeslet.so`` (hand-written HIP, C ABI in
``include/stokeslet.h``).  This package is its binding: ``_binding`` mirrors the C entry points
under the same names; the helpers below only marshal torch tensors (device memory and the
current stream) into those calls.
"""
from __future__ import annotations

from . import _binding
from ._binding import (EXPORTED, SL_EBUSY, SL_EHIP, SL_EINVAL, SL_ENOMEM, SL_ENOTFOUND, SL_ETIMEDOUT,
                       SL_FP64, SL_MIXED, SL_OK, SL_PARAM_KERNEL_TIMING, SL_PARAM_RHO64,
                       SL_PARAM_TARGETS_PER_LANE, SL_PARAM_WAVES_PER_SIMD, SlError, check, load, sl_create,
                       sl_destroy, sl_eval, sl_eval_fmm, sl_eval_noalloc, sl_eval_upsampled, sl_get_param, sl_get_stats, sl_last_error,
                       sl_patch_delta, sl_poll,
                       sl_request_bytes, sl_set_param, sl_submit, sl_surface_register,
                       sl_surface_release, sl_wait)

PRECISIONS = {"fp64": SL_FP64, "mixed": SL_MIXED}


def _soa(t, n_cols=3):
    """(n, 3) tensor -> contiguous (3, n) float64 tensor on the same device."""
    import torch
    t = t.to(torch.float64)
    return t.reshape(-1, n_cols).t().contiguous()


def _stream_handle(stream=None) -> int:
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return int(s.cuda_stream)


class Context:
    """Owns an ``sl_ctx`` on one device."""

    def __init__(self, device: int = 0, hbm_budget_bytes: int = 0):
        self.device = device
        self.ptr = sl_create(device, hbm_budget_bytes)

    def close(self):
        if self.ptr is not None and self.ptr.value:
            sl_destroy(self.ptr)
        self.ptr = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_rho64(self, value: float):
        check(sl_set_param(self.ptr, SL_PARAM_RHO64, value), "sl_set_param")

    def single_layer(self, X, w, f, delta, mu=1.0, targets=None, delta_tgt=None,
                     precision="fp64", stream=None, out=None):
        """u (n_tgt, 3) float64 on the device from torch device tensors X (N, 3), w (N,), f (N, 3).

        Enqueued on the current torch stream (or `stream`, which first waits for the current
        stream); returns without synchronizing.  The SoA copies are made on the stream the library
        works on, so the caching allocator does not hand their memory out before that work ends.
        """
        import torch
        prec = PRECISIONS[precision]
        cur = torch.cuda.current_stream()
        st_obj = cur if stream is None else stream
        if st_obj != cur:
            st_obj.wait_stream(cur)
        with torch.cuda.stream(st_obj):
            Xs, fs = _soa(X), _soa(f)
            ws = w.to(torch.float64).contiguous()
            n_src = Xs.shape[1]
            if targets is None:
                Ts, n_tgt, tp = None, n_src, (None, None, None)
            else:
                Ts = _soa(targets)
                n_tgt = Ts.shape[1]
                tp = (Ts[0].data_ptr(), Ts[1].data_ptr(), Ts[2].data_ptr())
            dts = None if delta_tgt is None else delta_tgt.to(torch.float64).contiguous()
            U = out if out is not None else torch.empty((3, n_tgt), dtype=torch.float64,
                                                        device=Xs.device)
            st = sl_eval(self.ptr, prec, n_src, Xs[0].data_ptr(), Xs[1].data_ptr(),
                         Xs[2].data_ptr(), ws.data_ptr(), fs[0].data_ptr(), fs[1].data_ptr(),
                         fs[2].data_ptr(), n_tgt, *tp, float(delta),
                         None if dts is None else dts.data_ptr(), float(mu), U[0].data_ptr(),
                         U[1].data_ptr(), U[2].data_ptr(), int(st_obj.cuda_stream))
        check(st, "sl_eval")
        return U.t()

    def patch_delta(self, X, n, C=1.0, stream=None, out=None):
        """Per-node delta = C delta* of eq. (regparam) (float64 device tensor of X.shape[0])
        for nodes X (n_patches n^2, 3) in patch-major, row-major order; enqueued on the current
        torch stream (or `stream`).  Pass the result as `delta_tgt` to single_layer."""
        import torch
        cur = torch.cuda.current_stream()
        st_obj = cur if stream is None else stream
        if st_obj != cur:
            st_obj.wait_stream(cur)
        with torch.cuda.stream(st_obj):
            Xs = _soa(X)
            npts = Xs.shape[1]
            if n < 1 or npts % (n * n) != 0:
                raise ValueError("X must hold whole patches of n x n nodes")
            D = out if out is not None else torch.empty(npts, dtype=torch.float64,
                                                        device=Xs.device)
            st = sl_patch_delta(self.ptr, npts // (n * n), int(n), Xs[0].data_ptr(),
                                Xs[1].data_ptr(), Xs[2].data_ptr(), float(C), D.data_ptr(),
                                int(st_obj.cuda_stream))
        check(st, "sl_patch_delta")
        return D

    def single_layer_upsampled(self, X, W, f, n, psi_up, mu=1.0, C=1.0, factor=4,
                               precision="fp64", stream=None, out=None):
        """u (N, 3) at the nodes X (n_patches n^2, 3) through the upsampling step: I_d S[I_u f]
        on I_u X, with fine weights psi_up (I_u W) h_u^2 from the area element W (N,) at the
        nodes and the fine POU values psi_up (n_patches (factor n)^2,), and delta_u = C delta*.
        Enqueued like single_layer."""
        import torch
        cur = torch.cuda.current_stream()
        st_obj = cur if stream is None else stream
        if st_obj != cur:
            st_obj.wait_stream(cur)
        with torch.cuda.stream(st_obj):
            Xs, fs = _soa(X), _soa(f)
            npts = Xs.shape[1]
            if n < 1 or npts % (n * n) != 0:
                raise ValueError("X must hold whole patches of n x n nodes")
            Ws = W.to(torch.float64).contiguous()
            ps = psi_up.to(torch.float64).contiguous()
            U = out if out is not None else torch.empty((3, npts), dtype=torch.float64,
                                                        device=Xs.device)
            st = sl_eval_upsampled(self.ptr, PRECISIONS[precision], npts // (n * n), int(n),
                                   int(factor), Xs[0].data_ptr(), Xs[1].data_ptr(),
                                   Xs[2].data_ptr(), Ws.data_ptr(), ps.data_ptr(),
                                   fs[0].data_ptr(), fs[1].data_ptr(), fs[2].data_ptr(), float(C),
                                   float(mu), U[0].data_ptr(), U[1].data_ptr(), U[2].data_ptr(),
                                   int(st_obj.cuda_stream))
        check(st, "sl_eval_upsampled")
        return U.t()

    def single_layer_fmm(self, X, w, f, delta, mu=1.0, delta_tgt=None, k=100, p_edge=6,
                         max_iter=100, precision="fp64", stream=None, out=None, labels=False):
        """u (N, 3) at the nodes X (targets = sources) by the single-level FMM: k clusters,
        p_edge equivalent points per cube edge.  With labels=True also returns the cluster of
        each node (int32 device tensor).  Synchronizes `stream` once (after the clustering)."""
        import torch
        cur = torch.cuda.current_stream()
        st_obj = cur if stream is None else stream
        if st_obj != cur:
            st_obj.wait_stream(cur)
        with torch.cuda.stream(st_obj):
            Xs, fs = _soa(X), _soa(f)
            ws = w.to(torch.float64).contiguous()
            n = Xs.shape[1]
            dts = None if delta_tgt is None else delta_tgt.to(torch.float64).contiguous()
            U = out if out is not None else torch.empty((3, n), dtype=torch.float64, device=Xs.device)
            L = torch.empty(n, dtype=torch.int32, device=Xs.device) if labels else None
            st = sl_eval_fmm(self.ptr, PRECISIONS[precision], n, Xs[0].data_ptr(), Xs[1].data_ptr(),
                             Xs[2].data_ptr(), ws.data_ptr(), fs[0].data_ptr(), fs[1].data_ptr(),
                             fs[2].data_ptr(), float(delta), None if dts is None else dts.data_ptr(),
                             float(mu), int(k), int(p_edge), int(max_iter), U[0].data_ptr(),
                             U[1].data_ptr(), U[2].data_ptr(), None if L is None else L.data_ptr(),
                             int(st_obj.cuda_stream))
        check(st, "sl_eval_fmm")
        return (U.t(), L) if labels else U.t()

    # -- serving ---------------------------------------------------------------------------
    def register_surface(self, X, w, delta) -> int:
        """Copy nodes X (N, 3) and weights w (N,) into a resident surface; returns its handle."""
        import torch
        Xs = _soa(X)
        ws = w.to(torch.float64).contiguous()
        # the library copies on a stream of its own: the SoA copies must be complete first
        torch.cuda.current_stream().synchronize()
        st, h = sl_surface_register(self.ptr, Xs.shape[1], Xs[0].data_ptr(), Xs[1].data_ptr(),
                                    Xs[2].data_ptr(), ws.data_ptr(), float(delta))
        check(st, "sl_surface_register")
        return h

    def release_surface(self, handle: int):
        check(sl_surface_release(self.ptr, handle), "sl_surface_release")

    def request_bytes(self, handle: int, precision="mixed") -> int:
        """Device memory a request on this surface holds while admitted (its staging)."""
        st, b = sl_request_bytes(self.ptr, handle, PRECISIONS[precision])
        check(st, "sl_request_bytes")
        return b

    def submit(self, handle: int, f, mu=1.0, precision="mixed", out=None):
        """Queue u = S[f] on a resident surface; returns (request id, (3, N) output tensor).

        The density copy and the output are kept alive here until the request is reported done.
        """
        import torch
        fs = _soa(f)
        U = out if out is not None else torch.empty_like(fs)
        torch.cuda.current_stream().synchronize()    # fs / U are ready before the device reads them
        st, rid = sl_submit(self.ptr, handle, PRECISIONS[precision], fs[0].data_ptr(),
                            fs[1].data_ptr(), fs[2].data_ptr(), float(mu), U[0].data_ptr(),
                            U[1].data_ptr(), U[2].data_ptr())
        check(st, "sl_submit")
        self._inflight = getattr(self, "_inflight", {})
        self._inflight[rid] = (fs, U)
        return rid, U

    def submit_prepared(self, handle: int, fs, U, mu=1.0, precision="mixed") -> int:
        """sl_submit on ready (3, N) float64 device tensors (no copy, no synchronization);
        the caller keeps fs and U alive until the request is done."""
        st, rid = sl_submit(self.ptr, handle, PRECISIONS[precision], fs[0].data_ptr(),
                            fs[1].data_ptr(), fs[2].data_ptr(), float(mu), U[0].data_ptr(),
                            U[1].data_ptr(), U[2].data_ptr())
        check(st, "sl_submit")
        return rid

    def wait(self, rid: int, timeout_s: float = 60.0):
        """Block until request `rid` is done; returns its (N, 3) output if it was submitted with
        submit(), else None."""
        check(sl_wait(self.ptr, rid, timeout_s), "sl_wait")
        entry = getattr(self, "_inflight", {}).pop(rid, None)
        return entry[1].t() if entry else None

    def poll(self, rid: int) -> bool:
        st, done = sl_poll(self.ptr, rid)
        check(st, "sl_poll")
        if done:
            getattr(self, "_inflight", {}).pop(rid, None)
        return done

    def stats(self):
        return sl_get_stats(self.ptr)
