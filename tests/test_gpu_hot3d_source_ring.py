"""The hotspot 3D source ring: bit-exact against the FP32 oracle where its slots go stale.

In a pass of all K steps the 3D hotspot kernel forms q = fma(cp, p, k_amb) of a plane once and
keeps it for levels 2..K in an LDS ring of K - 1 planes.  A workgroup of the balanced launch
streams several column segments one after another, so at the start of each segment the ring
still holds the previous column's planes; those slots may only reach pipeline-fill planes,
which are never stored.  Few workgroups (nwork 2..7) force many segments per workgroup; T runs
full passes and a shorter last pass (which re-forms q per level), across every instantiated K.
"""
import numpy as np
import pytest

import oracle
import paper_1802_00438_amd as S
from workloads import SETS, HOTSPOT, uniform

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()


@pytest.mark.parametrize("shape", [(37, 70, 130), (9, 100, 260), (64, 49, 129)])
@pytest.mark.parametrize("k", [1, 2, 3, 4])
@pytest.mark.parametrize("nwork", [0, 2, 7])
def test_hotspot3d_source_ring_bit_exact(shape, k, nwork):
    cf = SETS["H3"]
    x0 = uniform(shape, 300.0, 350.0, 9600 + k)
    power = uniform(shape, 0.0, 0.5, 9601)
    tuning = {"variant": 2, "k": k}
    if nwork:
        tuning["nwork"] = nwork
    else:
        tuning["seg_len"] = 5  # short z-tiles: many pipeline fills per column
    T = 2 * k + 1
    plan = S.Plan(HOTSPOT, shape, tuning)
    try:
        x = dev(x0)
        plan.run(x, cf, T, dev(power))
        torch.cuda.synchronize()
        got = x.cpu().numpy()
    finally:
        plan.close()
    ref = oracle.forward(x0, cf, T, power=power, dtype=np.float32)
    bad = np.flatnonzero(got.ravel() != ref.ravel())
    assert bad.size == 0, (shape, k, nwork, bad.size, np.unravel_index(bad[0], shape))
