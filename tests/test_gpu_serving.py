"""Serving: resident surfaces, HBM-footprint admission and the continuously batched persistent
kernel.  Parity with the oracle, bit-identical results alone vs in a mix, admission under a
small budget, release/lookup errors and relaunch of the kernel after it idles out."""
import math
import time

import numpy as np
import pytest

from capsule_inputs import ELLIPSOID_SERVING, RBC, SPHERE, make_surface, sh_force

pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-12, "mixed": 1e-6}


def eps(u, ref):
    return float(np.max(np.abs(u - ref)) / np.max(np.abs(ref)))


def dev_t(a):
    import torch
    return torch.as_tensor(np.asarray(a, dtype=np.float64), device=torch.device("cuda", 0))


@pytest.fixture(scope="module")
def surfaces():
    out = []
    for k, (shape, n) in enumerate([(SPHERE, 10), (ELLIPSOID_SERVING, 17), (RBC, 28), (RBC, 6)]):
        s = make_surface(shape, n)
        out.append((s, sh_force(s.x0, 500 + k), 2 * math.pi / (n + 1)))
    return out


@pytest.fixture(scope="module")
def refs(surfaces):
    import oracle
    return [oracle.single_layer(s.X, s.w, f, d, mu=0.8) for s, f, d in surfaces]


@pytest.fixture()
def ctx():
    import paper_2310_13908_amd as P
    c = P.Context(0, hbm_budget_bytes=256 << 20)
    yield c
    c.close()


@pytest.mark.parametrize("precision,rho64", [("fp64", 0.0), ("mixed", 0.0), ("mixed", 1.0)])
def test_requests_match_oracle(ctx, surfaces, refs, precision, rho64):
    """Mixed runs without a double-precision zone (the default) and with rho64 = 1, which a
    request takes from the context when it is submitted."""
    ctx.set_rho64(rho64)
    hs = [ctx.register_surface(dev_t(s.X), dev_t(s.w), d) for s, f, d in surfaces]
    rids = [ctx.submit(h, dev_t(f), mu=0.8, precision=precision)[0]
            for h, (s, f, d) in zip(hs, surfaces)]
    for rid, ref in zip(rids, refs):
        u = ctx.wait(rid, 60.0).cpu().numpy()
        assert eps(u, ref) < TOL[precision]
    st = ctx.stats()
    assert st.requests_done == len(rids) and st.kernel_launches >= 1


def test_rho64_changed_after_registration(ctx, surfaces, refs):
    """A request takes rho64 when it is submitted, also for a surface registered before: with
    rho64 = 12 (every near pair within the double-precision zone, beyond the single-precision
    cut of 5 delta) set after registration, the result equals that of a surface registered with
    rho64 = 12 already set, bit for bit, and is closer to the oracle than with rho64 = 0."""
    s, f, d = surfaces[2]
    ref = refs[2]
    h0 = ctx.register_surface(dev_t(s.X), dev_t(s.w), d)
    rid, _ = ctx.submit(h0, dev_t(f), mu=0.8, precision="mixed")
    u_zero = ctx.wait(rid, 60.0).cpu().numpy()
    try:
        ctx.set_rho64(12.0)
        rid, _ = ctx.submit(h0, dev_t(f), mu=0.8, precision="mixed")
        u_late = ctx.wait(rid, 60.0).cpu().numpy()
        h1 = ctx.register_surface(dev_t(s.X), dev_t(s.w), d)
        rid, _ = ctx.submit(h1, dev_t(f), mu=0.8, precision="mixed")
        u_early = ctx.wait(rid, 60.0).cpu().numpy()
    finally:
        ctx.set_rho64(0.0)
    assert np.array_equal(u_late, u_early)
    assert eps(u_late, ref) < eps(u_zero, ref) and eps(u_late, ref) < TOL["mixed"]


def test_alone_equals_mixed_bitwise(ctx, surfaces):
    """The same request served alone and inside a burst of other requests gives identical bits."""
    s, f, d = surfaces[2]
    h = ctx.register_surface(dev_t(s.X), dev_t(s.w), d)
    others = [ctx.register_surface(dev_t(o.X), dev_t(o.w), od) for o, of, od in surfaces]
    for precision in ("fp64", "mixed"):
        rid, _ = ctx.submit(h, dev_t(f), mu=0.8, precision=precision)
        alone = ctx.wait(rid).cpu().numpy()
        burst = []
        for k in range(12):
            o, of, od = surfaces[k % len(surfaces)]
            burst.append(ctx.submit(others[k % len(surfaces)], dev_t(of * (1 + k)), mu=0.8,
                                    precision=("fp64", "mixed")[k % 2])[0])
            if k == 5:
                mid, _ = ctx.submit(h, dev_t(f), mu=0.8, precision=precision)
        mixed = ctx.wait(mid).cpu().numpy()
        for r in burst:
            ctx.wait(r)
        assert np.array_equal(alone, mixed)


@pytest.fixture(scope="module")
def split_case():
    """RBC n = 180 (N = 194,400, 3,040 source clusters): its pair items are split into seven
    pieces of uneven cluster ranges; the oracle on 384 sampled targets."""
    import oracle
    s = make_surface(RBC, 180)
    f = sh_force(s.x0, 909)
    d = 2 * math.pi / 181
    idx = np.sort(np.random.default_rng(4).choice(s.N, 384, replace=False))
    ref = oracle.single_layer(s.X, s.w, f, d, mu=0.8, targets=s.X[idx])
    return s, f, d, idx, ref


def test_split_request_matches_oracle_and_mix(ctx, surfaces, split_case):
    """A request large enough for split pair items: parity with the oracle on sampled targets in
    both precisions, and the same bits alone and inside a burst of small requests."""
    s, f, d, idx, ref = split_case
    h = ctx.register_surface(dev_t(s.X), dev_t(s.w), d)
    others = [ctx.register_surface(dev_t(o.X), dev_t(o.w), od) for o, of, od in surfaces]
    for precision in ("fp64", "mixed"):
        rid, _ = ctx.submit(h, dev_t(f), mu=0.8, precision=precision)
        alone = ctx.wait(rid, 60.0).cpu().numpy()
        assert eps(alone[idx], ref) < TOL[precision]
        burst = []
        for k in range(8):
            o, of, od = surfaces[k % len(surfaces)]
            burst.append(ctx.submit(others[k % len(surfaces)], dev_t(of * (1 + k)), mu=0.8,
                                    precision=("fp64", "mixed")[k % 2])[0])
            if k == 3:
                mid, _ = ctx.submit(h, dev_t(f), mu=0.8, precision=precision)
        in_mix = ctx.wait(mid, 60.0).cpu().numpy()
        for r in burst:
            ctx.wait(r, 60.0)
        assert np.array_equal(alone, in_mix)


def test_fragmented_arena_is_compacted():
    """First fit can leave the free bytes in pieces that each are too small for a request's
    staging although together they hold it: surfaces A, B, C fill a budget up to a tail smaller
    than C's staging, A (smaller than that staging too) is released, and a request on C must
    still be admitted (the idle and pending surfaces move down), with correct results on the moved
    surfaces."""
    import oracle
    import paper_2310_13908_amd as P
    shapes = [(RBC, 24), (SPHERE, 16), (ELLIPSOID_SERVING, 40)]
    data = []
    for k, (shape, n) in enumerate(shapes):
        sf = make_surface(shape, n)
        data.append((sf, sh_force(sf.x0, 700 + k), 2 * math.pi / (n + 1)))
    # sizes of the three surfaces and of C's staging, from a roomy context
    with P.Context(0, hbm_budget_bytes=64 << 20) as c:
        sizes = []
        for sf, f, d in data:
            before = int(c.stats().bytes_admitted)
            h = c.register_surface(dev_t(sf.X), dev_t(sf.w), d)
            sizes.append(int(c.stats().bytes_admitted) - before)
        staging = c.request_bytes(h, "mixed")
    a, b, cc = sizes
    assert a < staging
    tail = staging - a // 2 // 256 * 256
    with P.Context(0, hbm_budget_bytes=a + b + cc + tail) as c:
        hs = [c.register_surface(dev_t(sf.X), dev_t(sf.w), d) for sf, f, d in data]
        c.release_surface(hs[0])
        sf, f, d = data[2]
        rid, _ = c.submit(hs[2], dev_t(f), mu=0.8, precision="mixed")
        u = c.wait(rid, 60.0).cpu().numpy()
        ref = oracle.single_layer(sf.X, sf.w, f, d, mu=0.8)
        assert eps(u, ref) < TOL["mixed"]
        sf, f, d = data[1]
        rid, _ = c.submit(hs[1], dev_t(f), mu=0.8, precision="fp64")
        u = c.wait(rid, 60.0).cpu().numpy()
        ref = oracle.single_layer(sf.X, sf.w, f, d, mu=0.8)
        assert eps(u, ref) < TOL["fp64"]


def test_admission_under_small_budget(surfaces, refs):
    """Budget that holds the surfaces but only a couple of requests' staging at a time:
    every request still completes, correctly, and the admitted bytes stay within the budget."""
    import paper_2310_13908_amd as P
    s, f, d = surfaces[2]
    np_pad = ((s.N + 255) // 256) * 256
    surf_bytes = np_pad * (4 * 8 + 3 * 4 + 4) + np_pad // 64 * 32 + np_pad // 128 * 64 + 8 * 256
    with P.Context(0) as c0:                          # one request's staging, as the library sizes it
        stage = c0.request_bytes(c0.register_surface(dev_t(s.X), dev_t(s.w), d), "mixed")
    with P.Context(0, hbm_budget_bytes=surf_bytes + surf_bytes // 2) as c:
        c.register_surface(dev_t(s.X), dev_t(s.w), d)
        with pytest.raises(P.SlError) as ei:           # a second copy does not fit
            c.register_surface(dev_t(s.X), dev_t(s.w), d)
        assert ei.value.status == P.SL_EBUSY
    budget = surf_bytes + stage + stage // 5          # one request's staging at a time
    with P.Context(0, hbm_budget_bytes=budget) as c:
        h = c.register_surface(dev_t(s.X), dev_t(s.w), d)
        rids = [c.submit(h, dev_t(f * (k + 1)), mu=0.8, precision="mixed")[0] for k in range(8)]
        for k, rid in enumerate(rids):
            u = c.wait(rid, 120.0).cpu().numpy()
            assert eps(u, refs[2] * (k + 1)) < TOL["mixed"]
        st = c.stats()
        assert st.requests_done == 8
        assert st.bytes_admitted <= budget


def test_release_and_errors(ctx, surfaces, refs):
    import paper_2310_13908_amd as P
    s, f, d = surfaces[3]
    h = ctx.register_surface(dev_t(s.X), dev_t(s.w), d)
    rid, _ = ctx.submit(h, dev_t(f), mu=0.8, precision="fp64")
    ctx.release_surface(h)                       # in flight: memory returned after completion
    u = ctx.wait(rid).cpu().numpy()
    assert eps(u, refs[3]) < TOL["fp64"]
    with pytest.raises(P.SlError) as ei:
        ctx.submit(h, dev_t(f), mu=0.8)
    assert ei.value.status == P.SL_ENOTFOUND
    with pytest.raises(P.SlError) as ei:
        ctx.release_surface(h)
    assert ei.value.status == P.SL_ENOTFOUND
    assert P.sl_wait(ctx.ptr, rid, 1.0) == P.SL_ENOTFOUND          # already retired
    assert P.sl_poll(ctx.ptr, 987654321)[0] == P.SL_ENOTFOUND
    h2 = ctx.register_surface(dev_t(s.X), dev_t(s.w), d)
    with pytest.raises(P.SlError) as ei:
        ctx.submit(h2, dev_t(f), mu=-1.0)
    assert ei.value.status == P.SL_EINVAL


def test_timeout_then_completion(surfaces):
    """sl_wait with a zero timeout on fresh work reports SL_ETIMEDOUT; the request still
    completes and a later wait returns it."""
    import paper_2310_13908_amd as P
    s = make_surface(RBC, 90)
    f = sh_force(s.x0, 77)
    with P.Context(0, hbm_budget_bytes=512 << 20) as c:
        h = c.register_surface(dev_t(s.X), dev_t(s.w), 2 * math.pi / 91)
        rid, _ = c.submit(h, dev_t(f), precision="fp64")
        assert P.sl_wait(c.ptr, rid, 0.0) == P.SL_ETIMEDOUT
        c.wait(rid, 60.0)


def test_kernel_relaunch_after_idle(ctx, surfaces, refs):
    """The persistent kernel exits after ~20 ms without work; new work relaunches it."""
    s, f, d = surfaces[0]
    h = ctx.register_surface(dev_t(s.X), dev_t(s.w), d)
    rid, _ = ctx.submit(h, dev_t(f), mu=0.8, precision="mixed")
    ctx.wait(rid)
    n0 = ctx.stats().kernel_launches
    time.sleep(0.2)
    rid, _ = ctx.submit(h, dev_t(f), mu=0.8, precision="mixed")
    u = ctx.wait(rid).cpu().numpy()
    assert eps(u, refs[0]) < TOL["mixed"]
    assert ctx.stats().kernel_launches >= n0 + 1


def test_register_while_kernel_busy(ctx, surfaces, refs):
    """Registering a surface while requests run drains the persistent kernel, packs the surface
    and relaunches: the requests queued before and after the registration all complete and
    match the oracle."""
    (s0, f0, d0), (s2, f2, d2) = surfaces[2], surfaces[1]
    h0 = ctx.register_surface(dev_t(s0.X), dev_t(s0.w), d0)
    rids = [ctx.submit(h0, dev_t(f0), mu=0.8, precision="fp64")[0] for _ in range(4)]
    n0 = ctx.stats().kernel_launches
    h2 = ctx.register_surface(dev_t(s2.X), dev_t(s2.w), d2)   # while the requests above run
    rid2, _ = ctx.submit(h2, dev_t(f2), mu=0.8, precision="fp64")
    for rid in rids:
        assert eps(ctx.wait(rid, 60.0).cpu().numpy(), refs[2]) < TOL["fp64"]
    assert eps(ctx.wait(rid2, 60.0).cpu().numpy(), refs[1]) < TOL["fp64"]
    assert ctx.stats().kernel_launches >= n0


def test_request_bytes(ctx, surfaces):
    """The staging a request holds: positive, larger in mixed (single-precision copies too), and
    refused for an unknown handle."""
    import paper_2310_13908_amd as P
    s, f, d = surfaces[1]
    h = ctx.register_surface(dev_t(s.X), dev_t(s.w), d)
    b64 = ctx.request_bytes(h, "fp64")
    b32 = ctx.request_bytes(h, "mixed")
    assert 24 * s.N <= b64 < b32
    st, _ = P.sl_request_bytes(ctx.ptr, h + 1000, P.SL_FP64)
    assert st == P.SL_ENOTFOUND
    ctx.release_surface(h)
    st, _ = P.sl_request_bytes(ctx.ptr, h, P.SL_FP64)
    assert st == P.SL_ENOTFOUND
