"""2D passes whose row segments are shorter than the fused-step count.

On grids small enough that 2-row segments fit one round of waves the tuner may pick segments
of 2 rows, well below the 2K rows of halo each tile streams.  Every instantiated k with
segments of 1, 2 and 3 rows, in the diffusion and hotspot forms, must equal the FP32 oracle
bit for bit (T = 2k + 1: full passes and a shorter last one); the transposed step at such
segments is compared with the FP64 oracle.
"""
import numpy as np
import pytest

import oracle
import paper_1802_00438_amd as S
from workloads import SETS, DIFFUSION, HOTSPOT, uniform

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()


@pytest.mark.parametrize("shape", [(256, 256), (70, 300)])
@pytest.mark.parametrize("k", [4, 8, 12, 16])
@pytest.mark.parametrize("seg", [1, 2, 3])
@pytest.mark.parametrize("form,cset", [(DIFFUSION, "D2"), (HOTSPOT, "H2")])
def test_short_segments_forward_bit_exact(shape, k, seg, form, cset):
    cf = SETS[cset]
    x0 = uniform(shape, 300.0, 350.0, 9700 + k)
    power = uniform(shape, 0.0, 0.5, 9701) if form == HOTSPOT else None
    T = 2 * k + 1
    plan = S.Plan(form, shape, {"variant": 2, "k": k, "seg_len": seg})
    try:
        x = dev(x0)
        plan.run(x, cf, T, None if power is None else dev(power))
        torch.cuda.synchronize()
        got = x.cpu().numpy()
    finally:
        plan.close()
    ref = oracle.forward(x0, cf, T, power=power, dtype=np.float32)
    bad = np.flatnonzero(got.ravel() != ref.ravel())
    assert bad.size == 0, (shape, k, seg, form, bad.size, np.unravel_index(bad[0], shape))


@pytest.mark.parametrize("k", [4, 12])
@pytest.mark.parametrize("seg", [1, 2])
def test_short_segments_adjoint(k, seg):
    shape = (256, 256)
    cf = SETS["AH2"]
    cot = uniform(shape, 0.5, 1.5, 9800 + k)
    T = 2 * k + 1
    plan = S.Plan(HOTSPOT, shape, {"variant": 2, "k": k, "seg_len": seg})
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
        assert float(np.max(np.abs(got - ref) / np.abs(ref))) <= 1e-5
