"""GPU parity of the radius-r star adjoint (stencil_adjoint_star) against the CPU oracle's
scatter-form adjoint, in 2D and 3D, for every radius, and the dot-product identity between
the GPU forward and the GPU adjoint.

Both kernels are covered: one cell per thread (rows not a multiple of 4) and four cells per
lane with DPP neighbours.  The kernels gather where the oracle scatters, so the sums round in
another order: the bar is an elementwise relative error of 1e-5 against the FP64 oracle.  The cotangents are positive and
the weights non-negative, so every gradient entry stays away from zero and the elementwise
bound is meaningful.
"""
import numpy as np
import pytest

import oracle
import paper_1802_00438_amd as S
from workloads import SETS, STAR_SETS, STAR3_SETS, uniform

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL = 1e-5
SRC = (0.125, 2.0 ** -8, 80.0)


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()


def w2(r):
    if r == 1:
        cf = SETS["A2"]
        return np.array([cf[0], cf[1], cf[2], cf[4], cf[3]], dtype=np.float32)
    return STAR_SETS[r]


def weights(shape, r):
    return w2(r) if len(shape) == 2 else STAR3_SETS[r]


def maxrel(a, b):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    return float(np.max(np.abs(a - b) / np.maximum(np.abs(b), 1e-30)))


def gpu_adjoint(shape, r, lam, T, hot):
    plan = S.StarPlan(r, shape, {"variant": 2, "k": 1})
    try:
        gx = torch.empty(shape, device="cuda")
        gp = torch.empty(shape, device="cuda") if hot else None
        plan.adjoint(dev(lam), weights(shape, r), T, gx, gp, SRC if hot else None)
        torch.cuda.synchronize()
    finally:
        plan.close()
    return gx.cpu().numpy(), None if gp is None else gp.cpu().numpy()


# one cell per thread where rows are not whole 16-byte groups; four cells per lane where nx is
# a multiple of 4 (rows of 4, 8, across a 256-column wave boundary, 3D rows of 4, 256 and 516)
SHAPES = [(131, 257), (1, 33), (29, 1), (5, 7), (3, 1000), (9, 70, 130), (20, 1, 33), (1, 40, 37), (2, 3, 1),
          (12, 129, 61), (64, 4), (7, 8), (3, 260), (5, 33, 516), (2, 1, 4), (17, 9, 256)]


@pytest.mark.parametrize("shape", SHAPES)
@pytest.mark.parametrize("r", [1, 2, 3, 4])
def test_star_adjoint_matches_the_oracle(shape, r):
    lam = uniform(shape, 0.5, 1.5, 8000 + 10 * r + len(shape))
    w = weights(shape, r)
    for T in (0, 1, 6):
        for hot in (False, True):
            gx, gp = gpu_adjoint(shape, r, lam, T, hot)
            ref, refp = oracle.star_adjoint(lam, w, T, cp=SRC[0] if hot else None)
            assert maxrel(gx, ref) <= TOL, (shape, r, T, hot, maxrel(gx, ref))
            if hot:
                if T == 0:
                    assert np.all(gp == 0.0)
                else:
                    assert maxrel(gp, refp) <= TOL, (shape, r, T, maxrel(gp, refp))


@pytest.mark.parametrize("shape,r", [((300, 412), 2), ((40, 100, 90), 3), ((24, 64, 200), 4)])
def test_star_adjoint_dot_product_identity(shape, r):
    """<F^T(x), y> = <x, (adjoint)^T(y)> with the GPU forward (the temporal-blocked kernel at its
    tuned k) and the GPU adjoint, inner products in FP64."""
    x = uniform(shape, -1.0, 1.0, 8100 + r)
    y = uniform(shape, -1.0, 1.0, 8110 + r)
    w = weights(shape, r)
    T = 9
    xd = dev(x)
    plan = S.StarPlan(r, shape)
    try:
        plan.run(xd, w, T)
        gx = torch.empty(shape, device="cuda")
        plan.adjoint(dev(y), w, T, gx)
        torch.cuda.synchronize()
    finally:
        plan.close()
    lhs = float(np.dot(xd.cpu().numpy().astype(np.float64).ravel(), y.astype(np.float64).ravel()))
    rhs = float(np.dot(x.astype(np.float64).ravel(), gx.cpu().numpy().astype(np.float64).ravel()))
    assert abs(lhs - rhs) <= 1e-5 * max(abs(lhs), 1.0), (lhs, rhs)


def test_star_adjoint_larger_grid_all_cells():
    """A 1000 x 1000 grid over 20 steps, every cell against the oracle."""
    shape, r, T = (1000, 1000), 2, 20
    lam = uniform(shape, 0.5, 1.5, 8200)
    gx, gp = gpu_adjoint(shape, r, lam, T, True)
    ref, refp = oracle.star_adjoint(lam, w2(r), T, cp=SRC[0])
    assert maxrel(gx, ref) <= TOL and maxrel(gp, refp) <= TOL


def test_star_adjoint_rejections():
    shape = (6, 64, 80)
    plan = S.StarPlan(2, shape, {"variant": 2, "k": 1})
    try:
        c = dev(np.ones(shape))
        g = torch.empty(shape, device="cuda")
        w = STAR3_SETS[2]
        with pytest.raises(S.StencilError) as e:
            S.stencil_adjoint_star(plan.handle, c, w, None, 1, c, None)  # grad_x0 aliases the cotangent
        assert e.value.status == -1
        with pytest.raises(S.StencilError) as e:
            S.stencil_adjoint_star(plan.handle, c, w, None, 1, g, torch.empty(shape, device="cuda"))  # no src
        assert e.value.status == -1
        bad = w.copy()
        bad[3] = np.inf
        with pytest.raises(S.StencilError) as e:
            S.stencil_adjoint_star(plan.handle, c, bad, None, 1, g, None)
        assert e.value.status == -1
        with pytest.raises(ValueError):
            plan.adjoint(c, w, 1, torch.empty((6, 64, 81), device="cuda"))  # wrong shape
        with pytest.raises(ValueError):
            plan.adjoint(c, w, 1, g, torch.empty(shape, device="cuda"))  # grad_power without src
    finally:
        plan.close()
    normal = S.Plan(S.DIFFUSION, (64, 80), {"variant": 2, "k": 4, "seg_len": 16})
    try:
        c = dev(np.ones((64, 80)))
        with pytest.raises(S.StencilError) as e:
            S.stencil_adjoint_star(normal.handle, c, STAR_SETS[2], None, 1, torch.empty_like(c), None)
        assert e.value.status == -1
    finally:
        normal.close()
