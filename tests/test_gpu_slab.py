"""The slab pass with ghost faces (stencil_run_slab): one device's share of a grid cut into slabs
along the streamed axis.

Each slab carries copies of its neighbours' planes (rows in 2D) as ghost planes; one pass of
T <= ghost depth fused steps must leave the slab's interior equal, bit for bit, to T steps of
the whole grid (FP32 oracle), write nothing into dst's ghost planes, and clamp at faces that are
true grid faces.  A three-slab run with ghost exchanges between passes (what a multi-device
run does over its links) must reproduce the whole grid's result.
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


def slab_case(full, power, cf, T, z0, z1, g, form, tuning=None):
    """Slab [z0, z1) of `full` along axis 0 with g ghost planes per side (0 at a true face)."""
    n = full.shape[0]
    glo = min(g, z0)
    ghi = min(g, n - z1)
    a, b = z0 - glo, z1 + ghi
    src = dev(full[a:b])
    pw = dev(power[a:b]) if power is not None else None
    dst = torch.full_like(src, float("nan"))
    plan = S.Plan(form, src.shape, tuning)
    try:
        plan.run_slab(src, dst, cf, T, glo, ghi, pw)
        torch.cuda.synchronize()
    finally:
        plan.close()
    out = dst.cpu().numpy()
    ref = oracle.forward(full, cf, T, power=power, dtype=np.float32)[z0:z1]
    got = out[glo:glo + (z1 - z0)]
    assert np.array_equal(got, ref), (z0, z1, g, T, float(np.nanmax(np.abs(got - ref))))
    assert np.isnan(out[:glo]).all() and np.isnan(out[glo + (z1 - z0):]).all()


@pytest.mark.parametrize("T", [1, 3, 4])
@pytest.mark.parametrize("z0,z1", [(20, 45), (0, 30), (40, 70)])
def test_slab_3d_diffusion(T, z0, z1):
    full = uniform((70, 50, 130), 0.0, 1.0, 9300)
    slab_case(full, None, SETS["A3"], T, z0, z1, 4, DIFFUSION)


@pytest.mark.parametrize("tuning", [None, {"variant": 2, "k": 6}])
def test_slab_3d_diffusion_deep_ghosts(tuning):
    full = uniform((64, 72, 264), 0.0, 1.0, 9301)
    slab_case(full, None, SETS["D3"], 6, 17, 47, 6, DIFFUSION, tuning)


@pytest.mark.parametrize("T", [2, 4])
def test_slab_3d_hotspot(T):
    full = uniform((48, 40, 200), 300.0, 350.0, 9302)
    p = uniform((48, 40, 200), 0.0, 1e-3, 9303)
    slab_case(full, p, SETS["AH3"], T, 10, 30, 4, HOTSPOT)


@pytest.mark.parametrize("T", [1, 8, 16])
@pytest.mark.parametrize("z0,z1", [(100, 260), (0, 120), (200, 300)])
def test_slab_2d_diffusion(T, z0, z1):
    full = uniform((300, 700), 0.0, 1.0, 9304)
    slab_case(full, None, SETS["A2"], T, z0, z1, 16, DIFFUSION)


def test_slab_2d_hotspot_split_launch():
    # 69 x 15 edge-free tiles: the pass splits into an edge-free and a frame launch
    full = uniform((1600, 16384), 300.0, 350.0, 9305)
    p = uniform((1600, 16384), 0.0, 1e-3, 9306)
    slab_case(full, p, SETS["H2"], 12, 100, 1540, 12, HOTSPOT, {"variant": 2, "k": 12, "seg_len": 96})


@pytest.mark.parametrize("ndim", [2, 3])
def test_three_slabs_with_ghost_exchange_equal_the_whole_grid(ndim):
    """Three slabs, ghost planes of depth k, passes of k steps, exchanges between passes."""
    k, passes = 4, 5
    shape = (90, 40, 136) if ndim == 3 else (150, 520)
    cf = SETS["A3"] if ndim == 3 else SETS["A2"]
    full = uniform(shape, 0.0, 1.0, 9310 + ndim)
    n = shape[0]
    cuts = [0, 31, 58, n]
    slabs = []
    for i in range(3):
        z0, z1 = cuts[i], cuts[i + 1]
        glo = k if i > 0 else 0
        ghi = k if i < 2 else 0
        a = dev(full[z0 - glo:z1 + ghi])
        slabs.append({"z0": z0, "z1": z1, "glo": glo, "ghi": ghi, "a": a, "b": torch.empty_like(a),
                      "plan": S.Plan(DIFFUSION, a.shape, {"variant": 2, "k": k})})
    try:
        for _ in range(passes):
            for s in slabs:
                s["plan"].run_slab(s["a"], s["b"], cf, k, s["glo"], s["ghi"])
            for s in slabs:
                s["a"], s["b"] = s["b"], s["a"]
            # exchange: each ghost region receives the neighbour's outermost interior planes
            for i, s in enumerate(slabs):
                if s["glo"]:
                    lo = slabs[i - 1]
                    m = lo["z1"] - lo["z0"]
                    s["a"][:k].copy_(lo["a"][lo["glo"] + m - k:lo["glo"] + m])
                if s["ghi"]:
                    hi = slabs[i + 1]
                    m = s["z1"] - s["z0"]
                    s["a"][s["glo"] + m:].copy_(hi["a"][hi["glo"]:hi["glo"] + k])
        torch.cuda.synchronize()
        got = np.concatenate([s["a"].cpu().numpy()[s["glo"]:s["glo"] + s["z1"] - s["z0"]] for s in slabs])
    finally:
        for s in slabs:
            s["plan"].close()
    ref = oracle.forward(full, cf, k * passes, dtype=np.float32)
    assert np.array_equal(got, ref)


def test_slab_rejections():
    x = dev(uniform((20, 30, 64), 0.0, 1.0, 9320))
    y = torch.empty_like(x)
    cf = SETS["D3"]
    plan = S.Plan(DIFFUSION, x.shape, {"variant": 2, "k": 4})
    try:
        with pytest.raises(S.StencilError) as e:  # T beyond a ghost depth
            plan.run_slab(x, y, cf, 5, 4, 4)
        assert e.value.status == -1
        with pytest.raises(S.StencilError) as e:  # no interior plane left
            plan.run_slab(x, y, cf, 2, 10, 10)
        assert e.value.status == -1
        with pytest.raises(S.StencilError) as e:  # in place
            plan.run_slab(x, x, cf, 2, 4, 4)
        assert e.value.status == -1
        with pytest.raises(S.StencilError) as e:  # beyond one pass of the kernels
            plan.run_slab(x, y, cf, 7, 8, 8)
        assert e.value.status == -2
    finally:
        plan.close()
    plain = S.Plan(DIFFUSION, x.shape, {"variant": 1})
    try:
        with pytest.raises(S.StencilError) as e:
            plain.run_slab(x, y, cf, 1, 1, 1)
        assert e.value.status == -2
    finally:
        plain.close()
