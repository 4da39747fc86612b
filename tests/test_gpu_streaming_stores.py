"""Parity on grids just above the streaming-store threshold (fields above 128 MiB).

Plans whose field exceeds 128 MiB store the output of the 2D temporal-blocked kernel and of
the one-step kernels with the nontemporal hint (a raw buffer store over the row instead of a
plain vector store); every smaller grid in the other tests takes the plain store.  These grids
sit just above the threshold, small enough for the oracle to compare every cell:

* 2D 6144 x 5504 (33.8M cells): the temporal-blocked pass split into the interior and frame
  launches, an unsplit pass, and the one-step kernel, in diffusion and hotspot form;
* 3D 324 x 320 x 328 (34.0M cells): the one-step kernel, and beside it the temporal-blocked
  tile and balanced launches (plain stores) at the same size, in both forms;
* the adjoint sweeps (transposed steps) of both, in hotspot form, and the radius-2 transposed
  step (its output stores carry the hint too).

Forward results must equal the FP32 oracle bit for bit (same operations in the same order on
every cell); adjoint results are compared with the FP64 oracle within 1e-5 elementwise (the
kernels gather where the oracle scatters), on positive cotangents and non-negative weights so
that every entry stays away from zero.
"""
import numpy as np
import pytest

import oracle
import paper_1802_00438_amd as S
from workloads import SETS, DIFFUSION, HOTSPOT, uniform

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

SHAPE2 = (6144, 5504)
SHAPE3 = (324, 320, 328)
TOL = 1e-5


def test_shapes_cross_the_threshold():
    for shape in (SHAPE2, SHAPE3):
        assert int(np.prod(shape)) * 4 > 128 << 20
        assert shape[-1] % 4 == 0  # vector (and so streaming) stores in interior tiles


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()


def gpu_forward(x0, power, cf, T, form, tuning):
    plan = S.Plan(form, x0.shape, tuning)
    try:
        x = dev(x0)
        plan.run(x, cf, T, None if power is None else dev(power))
        torch.cuda.synchronize()
        return x.cpu().numpy()
    finally:
        plan.close()


def assert_bit_exact(got, ref, what):
    bad = np.flatnonzero(got.ravel() != ref.ravel())
    assert bad.size == 0, (what, bad.size, np.unravel_index(bad[0], got.shape))


@pytest.mark.parametrize("form,cset", [(DIFFUSION, "D2"), (HOTSPOT, "H2")])
@pytest.mark.parametrize("tuning,T", [({"variant": 2, "k": 12, "seg_len": 64}, 13),   # interior + frame launches
                                      ({"variant": 2, "k": 8, "seg_len": 600}, 9),    # one launch per pass
                                      ({"variant": 1}, 2)])                           # one step per launch
def test_streaming_2d_forward_bit_exact(form, cset, tuning, T):
    cf = SETS[cset]
    x0 = uniform(SHAPE2, 300.0, 350.0, 9100)
    power = uniform(SHAPE2, 0.0, 0.5, 9101) if form == HOTSPOT else None
    got = gpu_forward(x0, power, cf, T, form, tuning)
    ref = oracle.forward(x0, cf, T, power=power, dtype=np.float32)
    assert_bit_exact(got, ref, (form, tuning, T))


@pytest.mark.parametrize("form,cset", [(DIFFUSION, "D3"), (HOTSPOT, "H3")])
@pytest.mark.parametrize("tuning,T", [({"variant": 2, "k": 4, "seg_len": 81}, 9),   # tile launch
                                      ({"variant": 2, "k": 3, "nwork": 512}, 7),   # balanced launch
                                      ({"variant": 1}, 2)])
def test_streaming_3d_forward_bit_exact(form, cset, tuning, T):
    cf = SETS[cset]
    x0 = uniform(SHAPE3, 0.0, 1.0, 9200)
    power = uniform(SHAPE3, 0.0, 0.5, 9201) if form == HOTSPOT else None
    got = gpu_forward(x0, power, cf, T, form, tuning)
    ref = oracle.forward(x0, cf, T, power=power, dtype=np.float32)
    assert_bit_exact(got, ref, (form, tuning, T))


def maxrel(a, b):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    return float(np.max(np.abs(a - b) / np.maximum(np.abs(b), 1e-30)))


@pytest.mark.parametrize("shape,cset,tuning,T", [(SHAPE2, "AH2", {"variant": 2, "k": 8, "seg_len": 64}, 9),
                                                 (SHAPE2, "AH2", {"variant": 1}, 2),
                                                 (SHAPE3, "AH3", {"variant": 2, "k": 3}, 7),
                                                 (SHAPE3, "AH3", {"variant": 1}, 2)])
def test_streaming_adjoint(shape, cset, tuning, T):
    cf = SETS[cset]
    cot = uniform(shape, 0.5, 1.5, 9300 + len(shape))
    plan = S.Plan(HOTSPOT, shape, tuning)
    try:
        gx = torch.empty(shape, device="cuda")
        gp = torch.empty(shape, device="cuda")
        plan.adjoint(dev(cot), cf, T, gx, gp)
        torch.cuda.synchronize()
    finally:
        plan.close()
    rx, rp = oracle.adjoint(cot, cf, T, form=HOTSPOT)
    assert maxrel(gx.cpu().numpy(), rx) <= TOL
    assert maxrel(gp.cpu().numpy(), rp) <= TOL


def test_streaming_star_adjoint():
    """The radius-r transposed step on a 3D grid above the threshold (nontemporal stores of
    lambda_{t-1}), in the hotspot form, against the FP64 oracle's scatter-form adjoint."""
    from workloads import STAR3_SETS
    r, T = 2, 3
    src = (0.125, 2.0 ** -8, 80.0)
    lam = uniform(SHAPE3, 0.5, 1.5, 9350)
    plan = S.StarPlan(r, SHAPE3, {"variant": 2, "k": 1})
    try:
        gx = torch.empty(SHAPE3, device="cuda")
        gp = torch.empty(SHAPE3, device="cuda")
        plan.adjoint(dev(lam), STAR3_SETS[r], T, gx, gp, src)
        torch.cuda.synchronize()
    finally:
        plan.close()
    rx, rp = oracle.star_adjoint(lam, STAR3_SETS[r], T, cp=src[0])
    assert maxrel(gx.cpu().numpy(), rx) <= TOL
    assert maxrel(gp.cpu().numpy(), rp) <= TOL
