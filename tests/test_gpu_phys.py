"""GPU parity of the paper-literal hotspot forms against the CPU oracle.

* Hotspot 2D in Table 2's physical form (STENCIL_HOTSPOT_PHYS): the kernels evaluate the
  printed formula in its own order, so results must equal the FP32 oracle bit for bit, across
  every instantiated k, ragged shapes, both tile launches (single and split), the plain
  one-step kernel and checkpointed runs.
* Hotspot 3D with the ambient coefficient equal to c_a (Table 2's Hotspot 3D ambient term),
  coefficient set H3p, through the ordinary hotspot kernels.
"""
import numpy as np
import pytest

import oracle
import paper_1802_00438_amd as S
from workloads import SETS, HOTSPOT, HOTSPOT_PHYS, uniform

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL = 1e-5


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()


def maxrel(a, b):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    return float(np.max(np.abs(a - b) / np.maximum(np.abs(b), 1e-30)))


def check(x0, power, cset, T, form, tuning=None):
    cf = SETS[cset]
    x = dev(x0)
    plan = S.Plan(form, x0.shape, tuning)
    try:
        plan.run(x, cf, T, dev(power))
        torch.cuda.synchronize()
        used = plan.tuning
    finally:
        plan.close()
    got = x.cpu().numpy()
    ref = oracle.forward(x0, cf, T, power=power, form=form, dtype=np.float32)
    assert maxrel(got, ref) <= TOL, (x0.shape, cset, T, tuning, used)
    assert np.array_equal(got, ref), (x0.shape, cset, T, tuning, used, maxrel(got, ref))
    return got


@pytest.mark.parametrize("shape", [(131, 257), (64, 900), (1, 33), (29, 1), (5, 7), (97, 1001)])
@pytest.mark.parametrize("k", [4, 8, 12, 16])
def test_phys_forward_all_k(shape, k):
    x0 = uniform(shape, 300.0, 350.0, 6100 + k)
    p = uniform(shape, 0.0, 1e-3, 6101 + k)
    for T in sorted({1, k - 1, k, 2 * k + 3}):
        for cset in ("HP2", "HPr"):
            check(x0, p, cset, T, HOTSPOT_PHYS, {"variant": 2, "k": k, "seg_len": 50})


def test_phys_plain_variant_and_autotuned_plan():
    x0 = uniform((300, 412), 300.0, 350.0, 6201)
    p = uniform((300, 412), 0.0, 1e-3, 6202)
    check(x0, p, "HPr", 23, HOTSPOT_PHYS, {"variant": 1})
    check(x0, p, "HPr", 23, HOTSPOT_PHYS)  # model-ranked, timed tuner


@pytest.mark.parametrize("k", [4, 12])
def test_phys_split_launch(k):
    """Wide grid, short segments: interior and frame tiles run as two launches on two streams."""
    x0 = uniform((1500, 2060), 300.0, 350.0, 6300 + k)
    p = uniform((1500, 2060), 0.0, 1e-3, 6301 + k)
    for T in sorted({k, 2 * k + 3}):
        check(x0, p, "HPr", T, HOTSPOT_PHYS, {"variant": 2, "k": k, "seg_len": 8})


def test_phys_ambient_field_stays_exact():
    """Zero power and a field at TEMP_AMB: every difference is zero, the field stays exact."""
    x0 = np.full((200, 300), 80.0, dtype=np.float32)
    got = check(x0, np.zeros_like(x0), "HPr", 40, HOTSPOT_PHYS, {"variant": 2, "k": 12, "seg_len": 64})
    assert np.all(got == 80.0)


def test_phys_checkpointed_run():
    cf = SETS["HPr"]
    x0 = uniform((150, 260), 300.0, 350.0, 6401)
    p = uniform((150, 260), 0.0, 1e-3, 6402)
    x = dev(x0)
    plan = S.Plan(HOTSPOT_PHYS, x0.shape, {"variant": 2, "k": 8, "seg_len": 40})
    try:
        plan.run_ckpt(x, cf, 45, 10, dev(p))
        torch.cuda.synchronize()
    finally:
        plan.close()
    ref = oracle.forward(x0, cf, 45, power=p, form=HOTSPOT_PHYS, dtype=np.float32)
    assert np.array_equal(x.cpu().numpy(), ref)


def test_phys_rejections():
    with pytest.raises(S.StencilError) as e:
        S.Plan(HOTSPOT_PHYS, (8, 9, 10))
    assert e.value.status == -2  # UNSUPPORTED: the physical form is 2D
    plan = S.Plan(HOTSPOT_PHYS, (64, 64), {"variant": 2, "k": 4, "seg_len": 16})
    try:
        g = dev(np.ones((64, 64)))
        with pytest.raises(S.StencilError) as e:
            plan.adjoint(g, SETS["HPr"], 3, torch.empty_like(g))
        assert e.value.status == -2
        with pytest.raises(S.StencilError) as e:
            plan.run(g, SETS["HPr"], 3, None)
        assert e.value.status == -1  # INVALID_ARG: needs a power map
    finally:
        plan.close()


@pytest.mark.parametrize("shape", [(6, 6, 6), (17, 45, 131), (9, 150, 400), (1, 60, 61)])
@pytest.mark.parametrize("k", [1, 2, 3, 4])
def test_hotspot3d_ambient_coefficient_equal_to_ca(shape, k):
    x0 = uniform(shape, 300.0, 350.0, 6500 + k)
    p = uniform(shape, 0.0, 1e-3, 6501 + k)
    for T in sorted({1, k, 2 * k + 1}):
        check(x0, p, "H3p", T, HOTSPOT, {"variant": 2, "k": k})
