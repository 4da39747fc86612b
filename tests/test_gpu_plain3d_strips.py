"""Parity of the one-step 3D kernel at every strip length the host picks.

The one-step 3D kernel marches a strip of planes per wave; the host takes the longest strip of
16, 32, ..., 256 planes that divides nz and still gives at least 16 workgroups per CU (4096 on
256 CUs; a workgroup is one 256-column chunk of one row and one strip), else 32 planes with a
shorter last strip.  Narrow grids (one chunk per row) reach each length at a size the oracle
compares cell by cell:

  (256, 4096, 4)   256 planes      (128, 4096, 8)  128 planes
  (192, 2048, 4)    64 planes      (48, 1400, 40)   16 planes
  (100, 64, 300)    32 planes, last strip 4 planes  (two chunks per row, a partial one)

Forward steps in both forms must equal the FP32 oracle bit for bit; the transposed step (the
adjoint, with grad_p) is compared with the FP64 oracle within 1e-5 elementwise on positive
cotangents.
"""
import numpy as np
import pytest

import oracle
import paper_1802_00438_amd as S
from workloads import SETS, DIFFUSION, HOTSPOT, uniform

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

SHAPES = [(256, 4096, 4), (128, 4096, 8), (192, 2048, 4), (48, 1400, 40), (100, 64, 300)]


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()


@pytest.mark.parametrize("shape", SHAPES)
@pytest.mark.parametrize("form,cset", [(DIFFUSION, "D3"), (HOTSPOT, "H3")])
def test_plain3d_strips_forward_bit_exact(shape, form, cset):
    cf = SETS[cset]
    x0 = uniform(shape, 0.0, 1.0, 9400 + shape[0])
    power = uniform(shape, 0.0, 0.5, 9401) if form == HOTSPOT else None
    T = 3
    plan = S.Plan(form, shape, {"variant": 1})
    try:
        x = dev(x0)
        plan.run(x, cf, T, None if power is None else dev(power))
        torch.cuda.synchronize()
        got = x.cpu().numpy()
    finally:
        plan.close()
    ref = oracle.forward(x0, cf, T, power=power, dtype=np.float32)
    bad = np.flatnonzero(got.ravel() != ref.ravel())
    assert bad.size == 0, (shape, form, bad.size, np.unravel_index(bad[0], shape))


def maxrel(a, b):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    return float(np.max(np.abs(a - b) / np.maximum(np.abs(b), 1e-30)))


@pytest.mark.parametrize("shape", SHAPES)
def test_plain3d_strips_adjoint(shape):
    cf = SETS["AH3"]
    cot = uniform(shape, 0.5, 1.5, 9500 + shape[0])
    T = 3
    plan = S.Plan(HOTSPOT, shape, {"variant": 1})
    try:
        gx = torch.empty(shape, device="cuda")
        gp = torch.empty(shape, device="cuda")
        plan.adjoint(dev(cot), cf, T, gx, gp)
        torch.cuda.synchronize()
    finally:
        plan.close()
    rx, rp = oracle.adjoint(cot, cf, T, form=HOTSPOT)
    assert maxrel(gx.cpu().numpy(), rx) <= 1e-5
    assert maxrel(gp.cpu().numpy(), rp) <= 1e-5
