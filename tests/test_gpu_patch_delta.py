"""The per-patch regularization parameter of Sec. 3.4, eq. (regparam), through the C ABI:
bit-exact against the oracle's plain loop over the definition, and the single layer evaluated
with it (delta_tgt) against the oracle to the parity tolerances."""
import math

import numpy as np
import pytest

from capsule_inputs import ELLIPSOID_PAPER, RBC, SPHERE, make_surface, sh_force

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


def gpu_patch_delta(ctx, X, n, C=1.0):
    import torch
    D = ctx.patch_delta(dev(X), n, C=C)
    torch.cuda.synchronize()
    return D.cpu().numpy()


@pytest.mark.parametrize("shape,n,C", [(SPHERE, 18, 1.0), (RBC, 64, 1.0), (ELLIPSOID_PAPER, 33, 2.5),
                                       (RBC, 2, 1.0), (RBC, 3, 0.5), (RBC, 200, 1.0)])
def test_bit_exact_against_the_oracle(ctx, shape, n, C):
    """Six patches of n x n nodes, n from the smallest patch with neighbours (2) to 240,000 nodes;
    every node's delta equal to the oracle's bit for bit."""
    import oracle
    s = make_surface(shape, n)
    d = gpu_patch_delta(ctx, s.X, n, C)
    ref = oracle.patch_delta(s.X, n, C=C)
    assert np.array_equal(d, ref)
    assert np.all(d > 0)


def test_single_patch_closed_form(ctx):
    """One flat patch with x = l^2, y = l': delta* is the diagonal of the last cell."""
    n = 37
    l, lp = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    X = np.stack([(l ** 2).ravel(), lp.ravel(), np.zeros(n * n)], axis=1).astype(np.float64)
    d = gpu_patch_delta(ctx, X, n)
    assert np.all(d == math.sqrt((2 * n - 3) ** 2 + 1.0))


def test_rejected_arguments(ctx):
    import torch
    import paper_2310_13908_amd as P
    X = dev(make_surface(RBC, 4).X)
    with pytest.raises(P.SlError) as e:
        ctx.patch_delta(X[:6], 1)                 # one node per patch: no neighbours
    assert e.value.status == P.SL_EINVAL
    with pytest.raises(P.SlError):
        ctx.patch_delta(X, 4, C=0.0)
    with pytest.raises(P.SlError):
        ctx.patch_delta(X, 4, C=float("nan"))
    Xs = X.t().contiguous()                       # output overlapping the x coordinates
    with pytest.raises(P.SlError) as e:
        P.check(P.sl_patch_delta(ctx.ptr, 6, 4, Xs[0].data_ptr(), Xs[1].data_ptr(),
                                 Xs[2].data_ptr(), 1.0, Xs[0].data_ptr(), 0), "sl_patch_delta")
    assert "aliases" in str(e.value)
    torch.cuda.synchronize()


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("shape,n", [(RBC, 24), (ELLIPSOID_PAPER, 16), (RBC, 64)])
def test_single_layer_with_patch_delta(ctx, shape, n, precision):
    """u = S^delta[f] with delta = delta*_i per patch (the paper's default rule, C = 1): the
    device delta fed to sl_eval, against the oracle with the oracle's delta; every target."""
    import torch
    import oracle
    s = make_surface(shape, n)
    f = sh_force(s.x0, 40 + n)
    X = dev(s.X)
    D = ctx.patch_delta(X, n)
    u = ctx.single_layer(X, dev(s.w), dev(f), 0.0, delta_tgt=D, precision=precision)
    torch.cuda.synchronize()
    dref = oracle.patch_delta(s.X, n)
    ref = oracle.single_layer(s.X, s.w, f, 0.0, delta_tgt=dref)
    u = u.cpu().numpy()
    assert float(np.max(np.abs(u - ref)) / np.max(np.abs(ref))) < TOL[precision]
