"""GPU parity of the paper-literal hotspot forms against the CPU oracle.

* The adjoint of the physical form (its symmetric linear part as the transposed step) against
  the oracle's scatter adjoint, within max normwise error 1e-5.

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
            S.stencil_run_batched([S.BatchItem(HOTSPOT_PHYS, 2, 64, 64, 1, g.data_ptr(), g.data_ptr(),
                                               S.make_coeffs(SETS["HPr"]), 3)], None, None)
        assert e.value.status == -2  # UNSUPPORTED: no batched launch of the physical form
        with pytest.raises(ValueError):  # the binding refuses a hotspot run without power
            plan.run(g, SETS["HPr"], 3, None)
        with pytest.raises(S.StencilError) as e:  # and so does the C ABI underneath
            S.stencil_run(plan.handle, g, None, SETS["HPr"], 3)
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


# ------------------------------------------------------------------ adjoint of the physical form

def normrel(a, b):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


def gpu_phys_adjoint(g, cf, T, tuning=None):
    gg = dev(g)
    plan = S.Plan(HOTSPOT_PHYS, g.shape, tuning)
    try:
        gx = torch.empty_like(gg)
        gp = torch.empty_like(gg)
        plan.adjoint(gg, cf, T, gx, gp)
        torch.cuda.synchronize()
    finally:
        plan.close()
    return gx.cpu().numpy(), gp.cpu().numpy()


@pytest.mark.parametrize("shape", [(131, 257), (64, 300), (1, 33), (40, 1)])
@pytest.mark.parametrize("tuning", [{"variant": 1}, {"variant": 2, "k": 4, "seg_len": 30},
                                    {"variant": 2, "k": 8, "seg_len": 30}, {"variant": 2, "k": 12, "seg_len": 50}])
def test_phys_adjoint_matches_oracle(shape, tuning):
    """The oracle's adjoint is the literal scatter of each term's partial derivative; the
    library applies the symmetric linear part as a gather."""
    cf = SETS["HPr"]
    g = uniform(shape, -1.0, 1.0, 6601)
    for T in (1, 5, 13):
        gx, gp = gpu_phys_adjoint(g, cf, T, tuning)
        rx, rp = oracle.adjoint(g, cf, T, form=HOTSPOT_PHYS)
        assert normrel(gx, rx) <= TOL, (shape, tuning, T)
        assert normrel(gp, rp) <= TOL, (shape, tuning, T)


def test_phys_adjoint_split_launch_and_dot_product():
    """Split 2D passes, and the dot-product identity <A^T y, x> = <y, A x> with the library's
    forward (zero power, TEMP_AMB = 0: the linear part) and adjoint."""
    cf = SETS["HPr"].copy()
    cf[9] = 0.0  # TEMP_AMB
    shape = (1500, 2060)
    x = uniform(shape, 0.0, 1.0, 6602)
    y = uniform(shape, 0.0, 1.0, 6603)
    tuning = {"variant": 2, "k": 8, "seg_len": 8}
    for T in (1, 19):
        xx = dev(x)
        plan = S.Plan(HOTSPOT_PHYS, shape, tuning)
        try:
            plan.run(xx, cf, T, dev(np.zeros(shape, np.float32)))
            torch.cuda.synchronize()
        finally:
            plan.close()
        aty, _ = gpu_phys_adjoint(y, cf, T, tuning)
        a = float(np.vdot(aty.astype(np.float64), x.astype(np.float64)))
        b = float(np.vdot(y.astype(np.float64), xx.cpu().numpy().astype(np.float64)))
        assert abs(a - b) / max(abs(a), abs(b)) <= TOL, (T, a, b)
    rx, rp = oracle.adjoint(y, cf, 19, form=HOTSPOT_PHYS)
    gx, gp = gpu_phys_adjoint(y, cf, 19, tuning)
    assert normrel(gx, rx) <= TOL and normrel(gp, rp) <= TOL


def test_phys_autograd_with_recompute():
    """StencilFn with the physical form: gradients against the oracle's adjoint of the same
    cotangent, with checkpoints re-run and checked bit for bit during backward."""
    cf = SETS["HPr"]
    shape, T = (96, 200), 30
    x0 = uniform(shape, 300.0, 350.0, 6604)
    p = uniform(shape, 0.0, 1e-3, 6605)
    y = uniform(shape, 300.0, 350.0, 6606)
    xt = dev(x0).requires_grad_(True)
    pt = dev(p).requires_grad_(True)
    out = S.StencilFn.apply(xt, pt, cf, T, 6, 1, {"variant": 2, "k": 4, "seg_len": 32}, HOTSPOT_PHYS)
    loss = 0.5 * ((out - dev(y)) ** 2).sum()
    loss.backward()
    xT = oracle.forward(x0, cf, T, power=p, form=HOTSPOT_PHYS, dtype=np.float32)
    assert np.array_equal(out.detach().cpu().numpy(), xT)
    rx, rp = oracle.adjoint(xT.astype(np.float64) - y, cf, T, form=HOTSPOT_PHYS)
    assert normrel(xt.grad.cpu().numpy(), rx) <= TOL
    assert normrel(pt.grad.cpu().numpy(), rp) <= TOL


def test_phys_run_captured_in_a_graph():
    """The physical form's split 2D passes (two streams, fork/join) record into a HIP graph;
    every replay equals the same steps run eagerly."""
    cf = SETS["HPr"]
    shape, T = (1500, 2060), 27
    x0 = uniform(shape, 300.0, 350.0, 6701)
    p = dev(uniform(shape, 0.0, 1e-3, 6702))
    tuning = {"variant": 2, "k": 8, "seg_len": 8}
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        plan = S.Plan(HOTSPOT_PHYS, shape, tuning)
        ref_plan = S.Plan(HOTSPOT_PHYS, shape, tuning)
    try:
        x = dev(x0)
        y = dev(x0)
        with torch.cuda.stream(s):
            plan.run(x, cf, T, p)
            ref_plan.run(y, cf, T, p)
        s.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g, stream=s):
            plan.run(x, cf, T, p)
        for _ in range(3):
            g.replay()
            torch.cuda.synchronize()
            with torch.cuda.stream(s):
                ref_plan.run(y, cf, T, p)
            s.synchronize()
            assert torch.equal(x, y)
    finally:
        plan.close()
        ref_plan.close()
