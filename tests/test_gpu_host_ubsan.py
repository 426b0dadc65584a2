"""The library's host code under UndefinedBehaviorSanitizer, on the GPU.

libstokeslet_ubsan.so is the same library with its host code (argument checks, planning, the
serving runtime, the FMM's host steps) built with -fsanitize=undefined (device code unchanged;
`python -m paper_2310_13908_amd.build --host-ubsan`).  A child process loads it in place of the
plain build and runs every entry point, the error paths included; any sanitizer report fails the
test, and a small sum is checked against the oracle so that the variant is known to compute."""
import os
import subprocess
import sys
import textwrap

import pytest

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_2310_13908_amd", "libstokeslet_ubsan.so")

SCRIPT = textwrap.dedent("""
    import math
    import numpy as np
    import torch
    import oracle
    import paper_2310_13908_amd as P
    from capsule_inputs import RBC, SPHERE, make_surface, sh_force
    assert P._binding.LIB_PATH.endswith("libstokeslet_ubsan.so")
    dev = torch.device("cuda", 0)
    T = lambda a: torch.as_tensor(np.asarray(a, dtype=np.float64), device=dev)
    s = make_surface(RBC, 12)
    f = sh_force(s.x0, 3)
    d = 2 * math.pi / 13
    ref = oracle.single_layer(s.X, s.w, f, d)
    with P.Context(0, hbm_budget_bytes=256 << 20) as ctx:
        for prec in ("fp64", "mixed"):
            u = ctx.single_layer(T(s.X), T(s.w), T(f), d, precision=prec).cpu().numpy()
            e = np.max(np.abs(u - ref)) / np.max(np.abs(ref))
            assert e < (1e-12 if prec == "fp64" else 1e-6), (prec, e)
            ctx.single_layer(T(s.X), T(s.w), T(f), d, targets=T(s.X[:100] + 0.01), precision=prec)
            ctx.single_layer(T(s.X), T(s.w), T(f), d, delta_tgt=T(np.full(s.N, d)), precision=prec)
        D = ctx.patch_delta(T(s.X), 12)
        ctx.single_layer_upsampled(T(s.X), T(s.W), T(f), 12, T(np.ones(6 * 48 * 48)), factor=4)
        ctx.single_layer_fmm(T(s.X), T(s.w), T(f), d, k=8, p_edge=4)
        h = ctx.register_surface(T(s.X), T(s.w), d)
        b = ctx.request_bytes(h, "mixed")
        rid, _ = ctx.submit(h, T(f), precision="mixed")
        ctx.wait(rid, 60.0)
        rid, _ = ctx.submit(h, T(f), precision="fp64")
        ctx.wait(rid, 60.0)
        ctx.stats()
        ctx.release_surface(h)
        # error paths
        st, _ = P.sl_request_bytes(ctx.ptr, h + 99, P.SL_FP64)
        assert st == P.SL_ENOTFOUND
        assert P.sl_set_param(ctx.ptr, P.SL_PARAM_TARGETS_PER_LANE, 3.0) == P.SL_EINVAL
        assert P.sl_eval(ctx.ptr, 0, -1, None, None, None, None, None, None, None, 0, None, None,
                         None, 1.0, None, 1.0, None, None, None, None) == P.SL_EINVAL
        print("host ubsan: ok", flush=True)
""")


@pytest.mark.skipif(not os.path.exists(LIB), reason="libstokeslet_ubsan.so not built "
                    "(python -m paper_2310_13908_amd.build --host-ubsan)")
def test_host_code_under_ubsan():
    env = dict(os.environ, SL_LIB=LIB, UBSAN_OPTIONS="print_stacktrace=1", PYTHONPATH=ROOT)
    r = subprocess.run([sys.executable, "-c", SCRIPT], cwd=ROOT, env=env, capture_output=True,
                       text=True, timeout=300)
    report = r.stdout + r.stderr
    assert r.returncode == 0, report[-4000:]
    assert "runtime error" not in report, report[-4000:]
    assert "host ubsan: ok" in r.stdout
