"""The upsampling step of Sec. 3.4 through the C ABI (sl_eval_upsampled): parity with the oracle's
sandwich (scipy not-a-knot splines, the oracle's delta* and double loop) and the sphere's closed
form."""
import numpy as np
import pytest

from capsule_inputs import ELLIPSOID_PAPER, RBC, SPHERE, fine_pou, make_surface, sh_force

pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-12, "mixed": 1e-6}


@pytest.fixture(scope="module")
def ctx():
    import torch
    import paper_2310_13908_amd as P
    assert torch.cuda.is_available()
    c = P.Context(0)
    yield c
    c.close()


def dev(a):
    import torch
    return torch.as_tensor(np.asarray(a, dtype=np.float64), device=torch.device("cuda", 0))


def run(ctx, s, f, n, precision, mu=1.0, C=1.0, factor=4):
    import torch
    u = ctx.single_layer_upsampled(dev(s.X), dev(s.W), dev(f), n, dev(fine_pou(n, factor)), mu=mu,
                                   C=C, factor=factor, precision=precision)
    torch.cuda.synchronize()
    return u.cpu().numpy()


def eps(u, ref):
    return float(np.max(np.abs(u - ref)) / np.max(np.abs(ref)))


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("shape,n,factor,mu,C", [(SPHERE, 6, 4, 1.0, 1.0), (RBC, 8, 4, 0.7, 1.0),
                                                  (ELLIPSOID_PAPER, 12, 4, 1.0, 1.0),
                                                  (RBC, 4, 2, 1.0, 2.0), (RBC, 24, 4, 1.0, 1.0)])
def test_parity_with_the_oracle(ctx, shape, n, factor, mu, C, precision):
    """Every node against the oracle's sandwich; sizes from the smallest spline patch (n = 4) to
    N = 3,456 coarse / 55,296 fine nodes."""
    import oracle
    s = make_surface(shape, n)
    f = sh_force(s.x0, 60 + n)
    u = run(ctx, s, f, n, precision, mu=mu, C=C, factor=factor)
    ref = oracle.single_layer_upsampled(s.X, s.W, f, n, fine_pou(n, factor), mu=mu, C=C,
                                        factor=factor)
    assert eps(u, ref) < TOL[precision]


@pytest.fixture(scope="module")
def rbc40_two_patches():
    """RBC n = 40 (N = 9,600 coarse, N_up = 153,600 fine nodes): the oracle's fine sum for the fine
    targets of patches 1 and 4 only (2 x 25,600 targets against all 153,600 sources), splined
    back to those patches' coarse nodes.  A patch's coarse values depend only on its own fine
    values, so these are the oracle's values at those nodes."""
    import oracle
    from capsule_inputs import fine_grid
    n, factor = 40, 4
    nf = factor * n
    s = make_surface(RBC, n)
    f = sh_force(s.x0, 4040)
    psi = fine_pou(n, factor)
    tc, tf = fine_grid(n, factor)
    Xu, wu = oracle.upsampled_surface(s.X, s.W, n, psi, factor)
    fu = oracle.spline_resample(f, n, tc, tf)
    du = oracle.patch_delta(Xu, nf)
    refs = {}
    for p in (1, 4):
        fine = slice(p * nf * nf, (p + 1) * nf * nf)
        uu = oracle.single_layer(Xu, wu, fu, 0.0, targets=Xu[fine], delta_tgt=du[fine])
        refs[p] = oracle.spline_resample(uu, nf, tf, tc)
    return s, f, n, refs


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_parity_fine_grid_above_2_17(ctx, rbc40_two_patches, precision):
    """The fine grid above 2^17 targets, where the FP64 path switches to two targets per lane
    (with per-target delta): the device's full evaluation at the coarse nodes of two patches
    against the oracle, element by element."""
    s, f, n, refs = rbc40_two_patches
    u = run(ctx, s, f, n, precision)
    for p, ref in refs.items():
        got = u[p * n * n:(p + 1) * n * n]
        assert eps(got, ref) < TOL[precision], (p, eps(got, ref))


def test_sphere_uniform_traction(ctx):
    """Unit sphere, uniform traction e_z: 2/3 e_z at every node (Stokes drag), through the whole
    upsampling step on the device."""
    n = 12
    s = make_surface(SPHERE, n)
    f = np.tile([0.0, 0.0, 1.0], (s.N, 1))
    for precision in ("fp64", "mixed"):
        u = run(ctx, s, f, n, precision)
        assert np.abs(u - [0.0, 0.0, 2.0 / 3.0]).max() < 2e-5


def test_rejected_arguments(ctx):
    import paper_2310_13908_amd as P
    s = make_surface(RBC, 3)
    with pytest.raises(P.SlError) as e:                    # a not-a-knot spline needs 4 nodes
        run(ctx, s, sh_force(s.x0, 1), 3, "fp64")
    assert e.value.status == P.SL_EINVAL
    s = make_surface(RBC, 4)
    with pytest.raises(P.SlError):
        run(ctx, s, sh_force(s.x0, 1), 4, "fp64", factor=0)
    with pytest.raises(P.SlError):
        run(ctx, s, sh_force(s.x0, 1), 4, "fp64", C=-1.0)
