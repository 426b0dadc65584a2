"""sl_eval_noalloc (the entry point that allocates nothing) against sl_eval through the C ABI.

Both run on the GPU with the same inputs; the allocation-free call must give sl_eval's result to
the single-layer tolerances (1e-12 in FP64, 1e-6 in mixed, relative infinity norm), on calls in a
row whose sizes shrink (the scratch keeps the previous call's contents), including a size where the
work is split into fewer items to fit the scratch, and must reject a problem whose workspace does
not fit without enqueuing anything."""
import math

import numpy as np
import pytest

from capsule_inputs import RBC, make_surface, sh_force

pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-12, "mixed": 1e-6}


def eps(u, ref):
    return float(np.max(np.abs(u - ref)) / np.max(np.abs(ref)))


def call(P, ctx, fn, prec, X, w, F, delta, T=None, D=None):
    """One call of fn (sl_eval or sl_eval_noalloc) on SoA device tensors; returns (status, u)."""
    import torch
    n_src = X.shape[1]
    n_tgt = n_src if T is None else T.shape[1]
    U = torch.full((3, n_tgt), float("nan"), dtype=torch.float64, device=X.device)
    tp = (None, None, None) if T is None else (T[0].data_ptr(), T[1].data_ptr(), T[2].data_ptr())
    st = fn(ctx.ptr, P.PRECISIONS[prec], n_src, X[0].data_ptr(), X[1].data_ptr(), X[2].data_ptr(),
            w.data_ptr(), F[0].data_ptr(), F[1].data_ptr(), F[2].data_ptr(), n_tgt, *tp, delta,
            None if D is None else D.data_ptr(), 1.0, U[0].data_ptr(), U[1].data_ptr(),
            U[2].data_ptr(), int(torch.cuda.current_stream().cuda_stream))
    torch.cuda.synchronize()
    return st, U.t().cpu().numpy()


def soa(a):
    import torch
    return torch.as_tensor(np.ascontiguousarray(np.asarray(a, dtype=np.float64).T),
                           device=torch.device("cuda", 0))


def test_noalloc_matches_sl_eval_on_shrinking_calls():
    import torch
    import paper_2310_13908_amd as P
    with P.Context(0) as ctx:
        cases = []
        # 701,784 points in FP64: the default split (12 ways per target block) needs more than the
        # 256 MiB scratch, so the allocation-free call runs 11; then C2 in both precisions; then a
        # small surface with distinct targets and per-target delta
        s = make_surface(RBC, 342)
        cases.append(("fp64", s, sh_force(s.x0, 342), 2 * math.pi / 343, None, None))
        s = make_surface(RBC, 64)
        f = sh_force(s.x0, 64)
        cases.append(("mixed", s, f, 2 * math.pi / 65, None, None))
        cases.append(("fp64", s, f, 2 * math.pi / 65, None, None))
        s = make_surface(RBC, 21)
        d = 2 * math.pi / 22
        T = s.X[::3] * 1.01
        dt = d * (0.6 + 0.8 * np.random.default_rng(21).random(T.shape[0]))
        for prec in ("fp64", "mixed"):
            cases.append((prec, s, sh_force(s.x0, 21), d, T, dt))
        for prec, s, f, d, T, dt in cases:
            print(f"[no-alloc] {prec} N={s.N} targets={'sources' if T is None else len(T)}", flush=True)
            X, F = soa(s.X), soa(f)
            w = torch.as_tensor(s.w, device=X.device)
            Td = None if T is None else soa(T)
            Dd = None if dt is None else torch.as_tensor(dt, device=X.device)
            st, ref = call(P, ctx, P.sl_eval, prec, X, w, F, d, Td, Dd)
            assert st == P.SL_OK
            st, u = call(P, ctx, P.sl_eval_noalloc, prec, X, w, F, d, Td, Dd)
            assert st == P.SL_OK, P.sl_last_error()
            assert np.all(np.isfinite(u))
            assert eps(u, ref) < TOL[prec], (prec, s.N, eps(u, ref))
            st, u2 = call(P, ctx, P.sl_eval_noalloc, prec, X, w, F, d, Td, Dd)
            assert st == P.SL_OK and np.array_equal(u, u2)


def test_noalloc_rejects_a_workspace_beyond_the_scratch():
    """2,000,000 points in mixed precision need about 300 MB of workspace even as one work item per
    target block: SL_EINVAL with a message, and the output untouched.  The buffers are real and of
    the stated size, so nothing could be read out of bounds."""
    import torch
    import paper_2310_13908_amd as P
    n = 2_000_000
    rng = np.random.default_rng(5)
    dev = torch.device("cuda", 0)
    X = torch.as_tensor(rng.standard_normal((3, n)), device=dev)
    F = torch.as_tensor(rng.standard_normal((3, n)), device=dev)
    w = torch.full((n,), 1e-6, dtype=torch.float64, device=dev)
    with P.Context(0) as ctx:
        st, u = call(P, ctx, P.sl_eval_noalloc, "mixed", X, w, F, 0.01)
        assert st == P.SL_EINVAL
        msg = P.sl_last_error()
        assert "scratch" in msg and "sl_eval_noalloc" in msg
        assert np.all(np.isnan(u))
