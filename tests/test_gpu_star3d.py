"""GPU parity of the radius-r 3D star stencils (stencil_create_star with ndim 3) against the
CPU oracle.

The kernel evaluates the oracle's FMA chain (cc; w_d and e_d by distance; the rows at y+d; the
rows at y-d; the planes at z-d; the planes at z+d), so results must equal the FP32 oracle bit
for bit, for every radius and instantiated k, on ragged shapes that span several 64 x 64
windows and z segments, grids thinner than the radius along any axis, passes shorter than k,
the one-step variant and the timed tuner.  At full size, sampled cells are checked against the
oracle on the sub-grid within r*T of them.
"""
import numpy as np
import pytest

import oracle
import paper_1802_00438_amd as S
from workloads import SETS, STAR3_SETS, STAR3_WORKLOAD, star3_field, uniform

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

KS3 = {1: [1, 2, 3], 2: [1, 2], 3: [1, 2], 4: [1]}


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()


def run_gpu(x0, r, T, tuning=None, weights=None):
    w = STAR3_SETS[r] if weights is None else weights
    x = dev(x0)
    plan = S.StarPlan(r, x0.shape, tuning)
    try:
        plan.run(x, w, T)
        torch.cuda.synchronize()
        used = plan.tuning
    finally:
        plan.close()
    return x.cpu().numpy(), used


def check(x0, r, T, tuning=None, weights=None):
    w = STAR3_SETS[r] if weights is None else weights
    got, used = run_gpu(x0, r, T, tuning, w)
    ref = oracle.star3d(x0, w, T, dtype=np.float32)
    if not np.array_equal(got, ref):
        d = np.abs(got.astype(np.float64) - ref)
        raise AssertionError((x0.shape, r, T, tuning, used, float(d.max()), np.argwhere(d > 0)[:4].tolist()))
    return got, used


# (nz, ny, nx): several windows in x and y with ragged last tiles, 1-wide axes, grids smaller
# than a window or than the radius
SHAPES = [(9, 70, 130), (20, 1, 33), (1, 40, 37), (5, 7, 9), (2, 3, 1), (12, 129, 61), (33, 64, 64)]


@pytest.mark.parametrize("shape", SHAPES)
@pytest.mark.parametrize("r", [1, 2, 3, 4])
def test_star3d_forward_all_k(shape, r):
    x0 = uniform(shape, 0.0, 1.0, 7500 + 10 * r)
    for k in KS3[r]:
        for T in sorted({1, max(1, k - 1), k, 2 * k + 1}):
            check(x0, r, T, {"variant": 2, "k": k, "seg_len": 4})


@pytest.mark.parametrize("r", [1, 2, 3, 4])
def test_star3d_segment_lengths(r):
    """Output planes split into z segments of every length from 1 to past nz."""
    x0 = uniform((17, 90, 100), 0.0, 1.0, 7550 + r)
    k = KS3[r][-1]
    for seg in (1, 2, 5, 16, 17, 40):
        check(x0, r, 2 * k + 1, {"variant": 2, "k": k, "seg_len": seg})


@pytest.mark.parametrize("r", [1, 2, 3, 4])
def test_star3d_one_step_variant_and_tuned_plan(r):
    x0 = uniform((40, 100, 90), 0.0, 1.0, 7600 + r)  # 360000 cells: the timed tuner runs
    check(x0, r, 5, {"variant": 1})
    _, used = check(x0, r, 7)
    assert used["k"] in KS3[r] and used["bsize_x"] == 64 and used["bsize_y"] == 64


def test_star3d_asymmetric_weights_need_every_term():
    """Weights with one non-zero neighbour term at a time: each term lands on its own axis,
    direction and distance (a transposed or misplaced term fails)."""
    r = 3
    x0 = uniform((14, 70, 75), 0.0, 1.0, 7650)
    for i in range(1, 1 + 6 * r):
        w = np.zeros(1 + 6 * r, np.float32)
        w[0] = 0.5
        w[i] = 0.5
        check(x0, r, 3, {"variant": 2, "k": 2, "seg_len": 5}, w)


def test_star3d_radius_one_equals_the_radius_one_form():
    """Radius 1 with the diffusion weights: the same cells as the radius-1 3D plan (whose chain
    is c, w, e, s, n, b, a), bit for bit."""
    cf = SETS["A3"]  # cc, cw, ce, cn, cs, cb, ca
    w = np.array([cf[0], cf[1], cf[2], cf[4], cf[3], cf[5], cf[6]], dtype=np.float32)  # cc, w, e, s, n, b, a
    x0 = uniform((21, 77, 140), 0.0, 1.0, 7660)
    got, _ = check(x0, 1, 9, {"variant": 2, "k": 3, "seg_len": 8}, w)
    x = dev(x0)
    plan = S.Plan(S.DIFFUSION, x0.shape, {"variant": 2, "k": 3})
    try:
        plan.run(x, cf, 9)
        torch.cuda.synchronize()
    finally:
        plan.close()
    assert np.array_equal(x.cpu().numpy(), got)


def test_star3d_rejections():
    g = dev(np.ones((6, 64, 80)))
    plan = S.StarPlan(2, (6, 64, 80), {"variant": 2, "k": 2, "seg_len": 4})
    try:
        with pytest.raises(ValueError):
            plan.run(g, STAR3_SETS[3], 1)  # 19 weights for radius 2
        bad = STAR3_SETS[2].copy()
        bad[11] = np.nan
        with pytest.raises(S.StencilError) as e:
            plan.run(g, bad, 1)
        assert e.value.status == -1
        with pytest.raises(S.StencilError) as e:
            S.stencil_run(plan.handle, g, None, SETS["D3"], 1)
        assert e.value.status == -1
    finally:
        plan.close()
    with pytest.raises(S.StencilError) as e:
        S.StarPlan(5, (6, 64, 80))
    assert e.value.status == -2


def test_star3d_run_captured_in_a_graph():
    """A 3D star run records into a HIP graph; every replay equals the same steps run eagerly."""
    r, T = 2, 5  # three passes at k = 2, the last one fusing one step
    x0 = uniform((30, 100, 120), 0.0, 1.0, 7700)
    w = STAR3_SETS[r]
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        plan = S.StarPlan(r, x0.shape, {"variant": 2, "k": 2, "seg_len": 8})
        ref_plan = S.StarPlan(r, x0.shape, {"variant": 2, "k": 2, "seg_len": 8})
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


def test_star3d_r2_512_full_size_samples():
    """The radius-2 3D workload at full size, auto-tuned as the bench runs it; each sampled cell
    against the FP32 oracle on the sub-grid within 2*T of it."""
    wl = STAR3_WORKLOAD
    x0 = star3_field(wl)
    r, T = wl["rad"], wl["T"]
    got, _ = run_gpu(x0, r, T)
    assert np.isfinite(got).all()
    n = wl["nx"]
    for idx in [(n // 2 + 3, n // 3 + 1, n // 5), (0, 0, 0), (n - 1, 17, n - 1), (250, n - 1, 3)]:
        sl = tuple(slice(max(0, i - r * T), min(n, i + r * T + 1)) for i in idx)
        ref = oracle.star3d(np.ascontiguousarray(x0[sl]), STAR3_SETS[r], T, dtype=np.float32)
        rv = ref[tuple(i - s.start for i, s in zip(idx, sl))]
        assert got[idx] == rv, (idx, got[idx], rv)
    # convex weights: the field stays within the bounds of the initial data
    assert got.min() >= x0.min() and got.max() <= x0.max()


SRC = (0.125, 2.0 ** -8, 80.0)  # cp, c_amb, t_amb


def w3_hot(r):
    """Radius-r 3D weights scaled to sum 7/8, so the source keeps the field bounded."""
    return (STAR3_SETS[r].astype(np.float64) * 0.875).astype(np.float32)


def check_hot3(x0, p, r, T, tuning=None):
    w = w3_hot(r)
    x = dev(x0)
    plan = S.StarPlan(r, x0.shape, tuning)
    try:
        plan.run(x, w, T, power=dev(p), src=SRC)
        torch.cuda.synchronize()
        used = plan.tuning
    finally:
        plan.close()
    got = x.cpu().numpy()
    ref = oracle.star3d(x0, w, T, dtype=np.float32, power=p, src=SRC)
    if not np.array_equal(got, ref):
        d = np.abs(got.astype(np.float64) - ref)
        raise AssertionError((x0.shape, r, T, tuning, used, float(d.max()), np.argwhere(d > 0)[:4].tolist()))


@pytest.mark.parametrize("shape", [(9, 70, 130), (20, 1, 33), (1, 40, 37), (2, 3, 1), (12, 129, 61)])
@pytest.mark.parametrize("r", [1, 2, 3, 4])
def test_star3d_hotspot_form_all_k(shape, r):
    """The 3D hotspot form bit for bit against the FP32 oracle, every radius and k."""
    x0 = uniform(shape, 300.0, 350.0, 7900 + 10 * r)
    p = uniform(shape, 0.0, 1.0, 7901 + 10 * r)
    for k in KS3[r]:
        for T in sorted({1, k, 2 * k + 1}):
            check_hot3(x0, p, r, T, {"variant": 2, "k": k, "seg_len": 5})


def test_star3d_hotspot_form_tuned_plan_and_a_graph():
    x0 = uniform((40, 100, 90), 300.0, 350.0, 7950)
    p = uniform((40, 100, 90), 0.0, 1.0, 7951)
    check_hot3(x0, p, 2, 7)  # timed tuner
    # a captured hotspot-form run replays like the eager one
    s = torch.cuda.Stream()
    w = w3_hot(2)
    with torch.cuda.stream(s):
        plan = S.StarPlan(2, x0.shape, {"variant": 2, "k": 2, "seg_len": 8})
    try:
        x, y, pd = dev(x0), dev(x0), dev(p)
        with torch.cuda.stream(s):
            plan.run(x, w, 5, power=pd, src=SRC)
            plan.run(y, w, 5, power=pd, src=SRC)
        s.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g, stream=s):
            plan.run(x, w, 5, power=pd, src=SRC)
        for _ in range(3):
            g.replay()
            torch.cuda.synchronize()
            with torch.cuda.stream(s):
                plan.run(y, w, 5, power=pd, src=SRC)
            s.synchronize()
            assert torch.equal(x, y)
    finally:
        plan.close()
