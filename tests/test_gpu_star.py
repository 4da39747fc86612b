"""GPU parity of the radius-r 2D star stencils (stencil_create_star / stencil_run_star) against
the CPU oracle.

The kernels evaluate the oracle's FMA chain (cc, then w_d and e_d by distance, then the rows
below, then the rows above), so results must equal the FP32 oracle bit for bit, for every
radius and instantiated k, on ragged and unaligned shapes, grids smaller than the radius, with
passes shorter than k, the one-step variant and the timed tuner.  At full size, sampled cells
are checked against the oracle on the sub-grid within r*T of them.
"""
import numpy as np
import pytest

import oracle
import paper_1802_00438_amd as S
from workloads import STAR_SETS, STAR_WORKLOAD, SETS, star_field, uniform

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL = 1e-5
KS = {1: [1, 2, 4, 8], 2: [1, 2, 4, 5, 8], 3: [1, 2, 4], 4: [1, 2, 4]}


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()


def maxrel(a, b):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    return float(np.max(np.abs(a - b) / np.maximum(np.abs(b), 1e-30)))


def weights(r):
    if r == 1:
        cf = SETS["A2"]  # cc, cw, ce, cn, cs -> cc, w1, e1, s1, n1
        return np.array([cf[0], cf[1], cf[2], cf[4], cf[3]], dtype=np.float32)
    return STAR_SETS[r]


def check(x0, r, T, tuning=None):
    w = weights(r)
    x = dev(x0)
    plan = S.StarPlan(r, x0.shape, tuning)
    try:
        plan.run(x, w, T)
        torch.cuda.synchronize()
        used = plan.tuning
    finally:
        plan.close()
    got = x.cpu().numpy()
    ref = oracle.star2d(x0, w, T, dtype=np.float32)
    assert maxrel(got, ref) <= TOL, (x0.shape, r, T, tuning, used)
    assert np.array_equal(got, ref), (x0.shape, r, T, tuning, used, maxrel(got, ref))
    return got


SHAPES = [(131, 257), (64, 900), (1, 33), (29, 1), (5, 7), (3, 3), (97, 1001), (300, 512)]


@pytest.mark.parametrize("shape", SHAPES)
@pytest.mark.parametrize("r", [1, 2, 3, 4])
def test_star_forward_all_k(shape, r):
    x0 = uniform(shape, 0.0, 1.0, 7100 + 10 * r)
    for k in KS[r]:
        for T in sorted({1, max(1, k - 1), k, 2 * k + 3}):
            check(x0, r, T, {"variant": 2, "k": k, "seg_len": 37})


@pytest.mark.parametrize("r", [1, 2, 3, 4])
def test_star_one_step_variant_and_tuned_plan(r):
    x0 = uniform((300, 412), 0.0, 1.0, 7200 + r)
    check(x0, r, 11, {"variant": 1})
    check(x0, r, 23)  # timed tuner (the grid has more than 2^16 cells)


def test_star_radius_one_equals_the_radius_one_kernel():
    x0 = uniform((257, 515), 0.0, 1.0, 7301)
    got = check(x0, 1, 29, {"variant": 2, "k": 8, "seg_len": 64})
    x = dev(x0)
    plan = S.Plan(S.DIFFUSION, x0.shape, {"variant": 2, "k": 8, "seg_len": 64})
    try:
        plan.run(x, SETS["A2"], 29)
        torch.cuda.synchronize()
    finally:
        plan.close()
    assert np.array_equal(x.cpu().numpy(), got)


def test_star_plans_reject_other_entry_points():
    g = dev(np.ones((64, 80)))
    plan = S.StarPlan(2, (64, 80), {"variant": 2, "k": 2, "seg_len": 16})
    try:
        with pytest.raises(S.StencilError) as e:
            S.stencil_run(plan.handle, g, None, SETS["D2"], 1)
        assert e.value.status == -1
        with pytest.raises(S.StencilError) as e:
            S.stencil_adjoint(plan.handle, g, None, SETS["D2"], 1, torch.empty_like(g), None, 0)
        assert e.value.status == -2
        with pytest.raises(ValueError):
            plan.run(g, STAR_SETS[3], 1)
        bad = STAR_SETS[2].copy()
        bad[3] = np.inf
        with pytest.raises(S.StencilError) as e:
            plan.run(g, bad, 1)
        assert e.value.status == -1
    finally:
        plan.close()
    normal = S.Plan(S.DIFFUSION, (64, 80), {"variant": 2, "k": 4, "seg_len": 16})
    try:
        with pytest.raises(S.StencilError) as e:
            S.stencil_run_star(normal.handle, g, STAR_SETS[2], 1)
        assert e.value.status == -1
    finally:
        normal.close()


def test_star2d_r2_16384_full_size_samples():
    """The radius-2 workload at full size, auto-tuned as the bench runs it; each sampled cell
    against the FP32 oracle on the sub-grid within 2*T of it."""
    wl = STAR_WORKLOAD
    x0 = star_field(wl)
    r, T = wl["rad"], wl["T"]
    x = dev(x0)
    plan = S.StarPlan(r, x0.shape)
    try:
        plan.run(x, STAR_SETS[r], T)
        torch.cuda.synchronize()
    finally:
        plan.close()
    got = x.cpu().numpy()
    assert np.isfinite(got).all()
    n = wl["nx"]
    for idx in [(n // 2 + 7, n // 3 + 1), (0, 0), (n - 1, 5000), (3000, n - 1)]:
        sl = tuple(slice(max(0, i - r * T), min(n, i + r * T + 1)) for i in idx)
        ref = oracle.star2d(np.ascontiguousarray(x0[sl]), STAR_SETS[r], T, dtype=np.float32)
        rv = ref[tuple(i - s.start for i, s in zip(idx, sl))]
        assert got[idx] == rv, (idx, got[idx], rv)
    # convex weights: the field stays within the bounds of the initial data
    assert got.min() >= x0.min() and got.max() <= x0.max()


def test_star_run_captured_in_a_graph():
    """stencil_run_star records into a HIP graph (its passes and the parity copy); every replay
    equals the same steps run eagerly, with eager work and synchronisation between replays."""
    r, T = 3, 9  # odd pass count with k = 2: the parity copy is in the graph too
    x0 = uniform((333, 700), 0.0, 1.0, 7401)
    w = STAR_SETS[r]
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        plan = S.StarPlan(r, x0.shape, {"variant": 2, "k": 2, "seg_len": 48})
        ref_plan = S.StarPlan(r, x0.shape, {"variant": 2, "k": 2, "seg_len": 48})
    try:
        x = dev(x0)
        y = dev(x0)
        with torch.cuda.stream(s):
            plan.run(x, w, T)
            ref_plan.run(y, w, T)
        s.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g, stream=s):
            plan.run(x, w, T)
        for _ in range(3):
            g.replay()
            torch.cuda.synchronize()
            with torch.cuda.stream(s):
                ref_plan.run(y, w, T)
            s.synchronize()
            assert torch.equal(x, y)
    finally:
        plan.close()
        ref_plan.close()


SRC = (0.125, 2.0 ** -8, 80.0)  # cp, c_amb, t_amb


def check_hot(x0, p, r, T, tuning=None, weights=None):
    w = weights if weights is not None else weights_for(r)
    x = dev(x0)
    plan = S.StarPlan(r, x0.shape, tuning)
    try:
        plan.run(x, w, T, power=dev(p), src=SRC)
        torch.cuda.synchronize()
        used = plan.tuning
    finally:
        plan.close()
    got = x.cpu().numpy()
    ref = oracle.star2d(x0, w, T, dtype=np.float32, power=p, src=SRC)
    assert np.array_equal(got, ref), (x0.shape, r, T, tuning, used, maxrel(got, ref))


def weights_for(r):
    """Radius-r weights scaled to sum 7/8, so the source keeps the field bounded."""
    return (weights(r).astype(np.float64) * 0.875).astype(np.float32)


@pytest.mark.parametrize("shape", [(131, 257), (1, 33), (29, 1), (5, 7), (97, 1001)])
@pytest.mark.parametrize("r", [1, 2, 3, 4])
def test_star_hotspot_form_all_k(shape, r):
    """The hotspot form (stencil_run_star_hotspot) bit for bit against the FP32 oracle."""
    x0 = uniform(shape, 300.0, 350.0, 7800 + 10 * r)
    p = uniform(shape, 0.0, 1.0, 7801 + 10 * r)
    for k in KS[r]:
        for T in sorted({1, k, 2 * k + 3}):
            check_hot(x0, p, r, T, {"variant": 2, "k": k, "seg_len": 37})


def test_star_hotspot_form_tuned_plan_and_rejections():
    x0 = uniform((300, 412), 300.0, 350.0, 7850)
    p = uniform((300, 412), 0.0, 1.0, 7851)
    check_hot(x0, p, 2, 13)  # timed tuner
    # a power map 4 bytes off 16-byte alignment takes the scalar path, same bits
    buf = torch.empty(p.size + 1, device="cuda")
    pv = buf[1:].view(p.shape)
    pv.copy_(dev(p))
    xa = dev(x0)
    pa = S.StarPlan(2, x0.shape, {"variant": 2, "k": 4, "seg_len": 64})
    try:
        pa.run(xa, weights_for(2), 9, power=pv, src=SRC)
        torch.cuda.synchronize()
    finally:
        pa.close()
    assert np.array_equal(xa.cpu().numpy(), oracle.star2d(x0, weights_for(2), 9, dtype=np.float32, power=p, src=SRC))
    g = dev(x0)
    plan = S.StarPlan(2, x0.shape, {"variant": 2, "k": 2, "seg_len": 32})
    try:
        with pytest.raises(ValueError):
            plan.run(g, weights_for(2), 1, power=dev(p))  # no src
        with pytest.raises(ValueError):
            plan.run(g, weights_for(2), 1, power=dev(p[:10]), src=SRC)  # wrong shape
        with pytest.raises(S.StencilError) as e:
            plan.run(g, weights_for(2), 1, power=dev(p), src=(0.1, float("nan"), 80.0))
        assert e.value.status == -1
        with pytest.raises(S.StencilError) as e:
            S.stencil_run_star_hotspot(plan.handle, g, g, weights_for(2), SRC, 1)  # power aliases grid
        assert e.value.status == -1
    finally:
        plan.close()
