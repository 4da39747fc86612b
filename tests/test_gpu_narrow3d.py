"""3D grids narrower than a window (fewer than 128 columns).

An even grid narrower than the 128-column window runs one window flush with x = 0: the lanes
past the row load its last two cells and idle, and the lane that holds x = nx passes on its left
neighbour's last cell so that cell nx - 1 reads its own value (the clamp).  Odd widths keep the
generic per-cell clamp.  Both must equal the FP32 oracle bit for bit, for every instantiated k,
in the tile and the balanced launch, with y windows flush with the grid edges (ny >= 48) and
crossing them (ny < 48); the transposed step (with grad_p) is compared with the FP64 oracle.
"""
import numpy as np
import pytest

import oracle
import paper_1802_00438_amd as S
from workloads import SETS, DIFFUSION, HOTSPOT, uniform

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

SHAPES = [(21, 60, 2), (13, 50, 4), (9, 97, 64), (17, 40, 120), (11, 130, 122), (8, 49, 126), (10, 70, 127),
          (6, 20, 94)]


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()


@pytest.mark.parametrize("shape", SHAPES)
@pytest.mark.parametrize("k", [1, 2, 3, 4])
@pytest.mark.parametrize("form,cset", [(DIFFUSION, "D3"), (HOTSPOT, "H3")])
@pytest.mark.parametrize("nwork", [0, 3])
def test_narrow3d_forward_bit_exact(shape, k, form, cset, nwork):
    cf = SETS[cset]
    x0 = uniform(shape, 300.0, 350.0, 9900 + shape[2])
    power = uniform(shape, 0.0, 0.5, 9901) if form == HOTSPOT else None
    tuning = {"variant": 2, "k": k}
    if nwork:
        tuning["nwork"] = nwork
    else:
        tuning["seg_len"] = 7
    T = 2 * k + 1
    plan = S.Plan(form, shape, tuning)
    try:
        x = dev(x0)
        plan.run(x, cf, T, None if power is None else dev(power))
        torch.cuda.synchronize()
        got = x.cpu().numpy()
    finally:
        plan.close()
    ref = oracle.forward(x0, cf, T, power=power, dtype=np.float32)
    bad = np.flatnonzero(got.ravel() != ref.ravel())
    assert bad.size == 0, (shape, k, form, nwork, bad.size, np.unravel_index(bad[0], shape))


@pytest.mark.parametrize("shape", SHAPES)
@pytest.mark.parametrize("k", [1, 3])
def test_narrow3d_adjoint(shape, k):
    cf = SETS["AH3"]
    cot = uniform(shape, 0.5, 1.5, 9950 + shape[2])
    T = 2 * k + 1
    plan = S.Plan(HOTSPOT, shape, {"variant": 2, "k": k, "seg_len": 7})
    try:
        gx = torch.empty(shape, device="cuda")
        gp = torch.empty(shape, device="cuda")
        plan.adjoint(dev(cot), cf, T, gx, gp)
        torch.cuda.synchronize()
    finally:
        plan.close()
    rx, rp = oracle.adjoint(cot, cf, T, form=HOTSPOT)
    for got, ref in ((gx, rx), (gp, rp)):
        got = got.cpu().numpy().astype(np.float64)
        assert float(np.max(np.abs(got - ref) / np.abs(ref))) <= 1e-5, (shape, k)
