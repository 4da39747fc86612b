"""GPU parity: the HIP library (through its C ABI) against the CPU oracle.

Bar (from the requirement): FP32 GPU results within max-rel 1e-5 of the FP32 oracle,
elementwise, on the same seeded inputs; the error against FP64 is reported.  Because every
kernel evaluates each cell update in the same fixed FMA order as the oracle, forward results
are also expected to be bit-identical to the FP32 oracle, which is asserted as well: it is
the sharpest check of halo, tail and boundary handling across tilings.
"""
import numpy as np
import pytest

import oracle
import paper_1802_00438_amd as S
from workloads import SETS, DIFFUSION, HOTSPOT, uniform

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL = 1e-5


def maxrel(a, b):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    return float(np.max(np.abs(a - b) / np.maximum(np.abs(b), 1e-30)))


def normrel(a, b):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()


def gpu_forward(x0, cf, T, power=None, tuning=None):
    form = HOTSPOT if power is not None else DIFFUSION
    x = dev(x0)
    p = dev(power) if power is not None else None
    plan = S.Plan(form, x0.shape, tuning)
    try:
        plan.run(x, cf, T, p)
        torch.cuda.synchronize()
        used = plan.tuning
    finally:
        plan.close()
    return x.cpu().numpy(), used


def check_forward(x0, cset, T, power=None, tuning=None, bitwise=True):
    cf = SETS[cset]
    got, used = gpu_forward(x0, cf, T, power, tuning)
    ref32 = oracle.forward(x0, cf, T, power=power, dtype=np.float32)
    ref64 = oracle.forward(x0, cf, T, power=power)
    assert maxrel(got, ref32) <= TOL, (x0.shape, cset, T, tuning, used)
    if bitwise:
        assert np.array_equal(got, ref32), (x0.shape, cset, T, tuning, used, maxrel(got, ref32))
    return maxrel(got, ref64)


# ------------------------------------------------------------------ forward 2D

SHAPES_2D = [(256, 256), (131, 257), (1, 300), (300, 1), (5, 7), (3, 1000), (700, 9), (67, 613)]


@pytest.mark.parametrize("shape", SHAPES_2D)
@pytest.mark.parametrize("k", [4, 8, 12, 16, 20, 24])
def test_forward_2d_diffusion_all_k(shape, k):
    x0 = uniform(shape, 0.0, 1.0, 1000 + k)
    for T in sorted({0, 1, k - 1, k, k + 1, 3 * k + 2}):
        check_forward(x0, "A2", T, tuning={"variant": 2, "k": k, "seg_len": 37})


@pytest.mark.parametrize("shape", [(131, 257), (64, 900), (1, 33), (29, 1)])
@pytest.mark.parametrize("k", [4, 8, 12, 16])
def test_forward_2d_hotspot_all_k(shape, k):
    x0 = uniform(shape, 300.0, 350.0, 2000 + k)
    p = uniform(shape, 0.0, 1e-3, 2001 + k)
    for T in sorted({1, k - 1, k, 2 * k + 3}):
        check_forward(x0, "H2", T, power=p, tuning={"variant": 2, "k": k, "seg_len": 50})
        check_forward(x0, "AH2", T, power=p, tuning={"variant": 2, "k": k, "seg_len": 50})


def test_forward_2d_small_workload_exact_config():
    """The 256x256, 16-step diffusion workload with auto-tuning, against both oracles."""
    x0 = uniform((256, 256), 0.0, 1.0, 1000)
    err64 = check_forward(x0, "D2", 16)
    assert err64 < 1e-6


@pytest.mark.parametrize("variant", [1, 2])
def test_forward_2d_plain_and_blocked_agree_bitwise(variant):
    x0 = uniform((190, 333), 0.0, 1.0, 77)
    check_forward(x0, "A2", 21, tuning={"variant": variant, "k": 8 if variant == 2 else 0})


def test_forward_2d_unaligned_width():
    # nx % 4 != 0 forces the scalar load/store path in every tile
    x0 = uniform((97, 1001), 0.0, 1.0, 78)
    check_forward(x0, "A2", 19, tuning={"variant": 2, "k": 8, "seg_len": 30})


# Passes with at least 1024 interior tiles run as two launches on two streams: the interior
# rectangle of tiles (edge-free kernel) and the frame of edge tiles.  These grids are wide
# and cut into short segments so the split is taken.

@pytest.mark.parametrize("k", [4, 12])
def test_forward_2d_split_launch(k):
    x0 = uniform((1500, 2060), 300.0, 350.0, 81 + k)
    p = uniform((1500, 2060), 0.0, 1e-3, 82 + k)
    for T in sorted({k, 2 * k + 3}):
        check_forward(x0, "AH2", T, power=p, tuning={"variant": 2, "k": k, "seg_len": 8})
        check_forward(x0, "A2", T, tuning={"variant": 2, "k": k, "seg_len": 8})


@pytest.mark.parametrize("k", [4, 8])
def test_adjoint_2d_split_launch(k):
    cf = SETS["AH2"]
    g = uniform((1500, 2060), -1.0, 1.0, 83 + k)
    for T in (k, 2 * k + 1):
        gx, gp = gpu_adjoint(g, cf, T, HOTSPOT, tuning={"variant": 2, "k": k, "seg_len": 8})
        rx, rp = oracle.adjoint(g, cf, T, form=HOTSPOT)
        assert normrel(gx, rx) <= TOL, (k, T)
        assert normrel(gp, rp) <= TOL, (k, T)


# ------------------------------------------------------------------ forward 3D

# The last three shapes take the edge-flush tiling of forward passes (first and last window
# of an axis flush with the grid edge): one window exactly the grid's size, two flush
# windows, and flush windows with ordinary tiles between them.
SHAPES_3D = [(6, 6, 6), (1, 40, 37), (20, 1, 33), (9, 70, 130), (33, 50, 129), (3, 2, 300), (40, 97, 5),
             (7, 48, 128), (11, 96, 256), (20, 150, 400)]


@pytest.mark.parametrize("shape", SHAPES_3D)
@pytest.mark.parametrize("k", [1, 2, 3, 4, 5, 6])
def test_forward_3d_diffusion_all_k(shape, k):
    x0 = uniform(shape, 0.0, 1.0, 3000 + k)
    for T in sorted({0, 1, k, k + 1, 3 * k + 2}):
        check_forward(x0, "A3", T, tuning={"variant": 2, "k": k, "seg_len": 7})


@pytest.mark.parametrize("shape", [(6, 6, 6), (17, 45, 131), (1, 60, 61), (5, 96, 256)])
@pytest.mark.parametrize("k", [1, 2, 3, 4])
def test_forward_3d_hotspot_all_k(shape, k):
    x0 = uniform(shape, 300.0, 350.0, 4000 + k)
    p = uniform(shape, 0.0, 1e-3, 4001 + k)
    for T in sorted({1, k, 2 * k + 1}):
        check_forward(x0, "H3", T, power=p, tuning={"variant": 2, "k": k, "seg_len": 6})
        check_forward(x0, "AH3", T, power=p, tuning={"variant": 2, "k": k, "seg_len": 6})


# With k given and no segment length, a 3D plan uses the balanced launch: every workgroup
# streams an equal share of (x-y column, plane) units, crossing column boundaries mid-share.

@pytest.mark.parametrize("shape", [(6, 6, 6), (9, 70, 130), (33, 50, 129), (3, 2, 300), (70, 40, 37),
                                   (20, 150, 400)])
@pytest.mark.parametrize("k", [1, 2, 3, 4, 5, 6])
def test_forward_3d_diffusion_balanced_launch(shape, k):
    x0 = uniform(shape, 0.0, 1.0, 3100 + k)
    for T in sorted({1, k, 2 * k + 1}):
        check_forward(x0, "A3", T, tuning={"variant": 2, "k": k})


@pytest.mark.parametrize("shape", [(17, 45, 131), (40, 97, 5), (9, 150, 400)])
@pytest.mark.parametrize("k", [1, 2, 3, 4])
def test_forward_3d_hotspot_balanced_launch(shape, k):
    x0 = uniform(shape, 300.0, 350.0, 4100 + k)
    p = uniform(shape, 0.0, 1e-3, 4101 + k)
    for T in sorted({1, k, 2 * k + 1}):
        check_forward(x0, "AH3", T, power=p, tuning={"variant": 2, "k": k})


@pytest.mark.parametrize("k", [1, 2, 3, 4])
def test_adjoint_3d_balanced_launch(k):
    cf = SETS["AH3"]
    g = uniform((21, 45, 131), -1.0, 1.0, 5100 + k)
    for T in (1, k + 1, 3 * k):
        gx, gp = gpu_adjoint(g, cf, T, HOTSPOT, tuning={"variant": 2, "k": k})
        rx, rp = oracle.adjoint(g, cf, T, form=HOTSPOT)
        assert normrel(gx, rx) <= TOL, (k, T)
        assert normrel(gp, rp) <= TOL, (k, T)


@pytest.mark.parametrize("shape,cset,form", [((24, 100, 260), "AH3", HOTSPOT), ((30, 64, 130), "A3", DIFFUSION),
                                             ((700, 1200), "AH2", HOTSPOT)])
def test_adjoint_autotuned_plan(shape, cset, form):
    """Auto-tuned plans time the adjoint's own candidates (k, segment, balanced launch in 3D);
    whichever wins must match the oracle."""
    cf = SETS[cset]
    g = uniform(shape, -1.0, 1.0, 5200)
    for T in (7, 16):
        gx, gp = gpu_adjoint(g, cf, T, form)
        rx, rp = oracle.adjoint(g, cf, T, form=form)
        assert normrel(gx, rx) <= TOL, (shape, T)
        if form == HOTSPOT:
            assert normrel(gp, rp) <= TOL, (shape, T)


def test_forward_3d_plain_variant():
    x0 = uniform((11, 23, 45), 0.0, 1.0, 79)
    check_forward(x0, "A3", 9, tuning={"variant": 1})


# ------------------------------------------------------------------ adjoint

def gpu_adjoint(g, cf, T, form, tuning=None, recompute=0, x0=None, power=None, ckpt_every=0):
    plan = S.Plan(form, g.shape, tuning)
    try:
        cot = dev(g)
        gx = torch.empty_like(cot)
        gp = torch.empty_like(cot) if form == HOTSPOT else None
        pw = dev(power) if power is not None else None
        if recompute:
            x = dev(x0)
            plan.run_ckpt(x, cf, T, ckpt_every, pw)
        plan.adjoint(cot, cf, T, gx, gp, pw, recompute)
        torch.cuda.synchronize()
    finally:
        plan.close()
    return gx.cpu().numpy(), (gp.cpu().numpy() if gp is not None else None)


@pytest.mark.parametrize("shape,cset,form", [((131, 257), "A2", DIFFUSION), ((64, 300), "AH2", HOTSPOT),
                                             ((1, 50), "AH2", HOTSPOT), ((40, 1), "A2", DIFFUSION),
                                             ((9, 70, 130), "A3", DIFFUSION), ((13, 45, 61), "AH3", HOTSPOT),
                                             ((1, 20, 30), "AH3", HOTSPOT), ((5, 1, 9), "A3", DIFFUSION)])
@pytest.mark.parametrize("variant,k2,k3", [(1, 0, 0), (2, 4, 1), (2, 8, 2), (2, 12, 3), (2, 12, 4)])
def test_adjoint_matches_oracle(shape, cset, form, variant, k2, k3):
    cf = SETS[cset]
    g = uniform(shape, -1.0, 1.0, 5000)
    for T in (1, 5, 13):
        gx, gp = gpu_adjoint(g, cf, T, form, tuning={"variant": variant, "k": k2 if len(shape) == 2 else k3,
                                                     "seg_len": 20})
        rx, rp = oracle.adjoint(g, cf, T, form=form)
        assert normrel(gx, rx) <= TOL, (shape, cset, T)
        if form == HOTSPOT:
            assert normrel(gp, rp) <= TOL, (shape, cset, T)


@pytest.mark.parametrize("shape,cset", [((77, 301), "A2"), ((15, 40, 140), "A3")])
def test_dot_product_identity_on_gpu(shape, cset):
    """<A^T y, x> = <y, A x> for the T-step linear map, FP64 inner products of GPU results."""
    cf = SETS[cset]
    x = uniform(shape, 0.0, 1.0, 6000)
    y = uniform(shape, 0.0, 1.0, 6001)
    T = 20
    Ax, _ = gpu_forward(x, cf, T, tuning={"variant": 2, "k": 8 if len(shape) == 2 else 3})
    ATy, _ = gpu_adjoint(y, cf, T, DIFFUSION)
    a = float(np.vdot(ATy.astype(np.float64), x.astype(np.float64)))
    b = float(np.vdot(y.astype(np.float64), Ax.astype(np.float64)))
    assert abs(a - b) / max(abs(a), abs(b)) <= 1e-5


def test_symmetric_adjoint_equals_forward():
    """Mirror-symmetric weights make the operator symmetric: the adjoint of the linear part is
    the forward map itself (checked against the oracle's forward)."""
    cf = SETS["D3"]
    g = uniform((20, 33, 65), 0.0, 1.0, 6100)
    gx, _ = gpu_adjoint(g, cf, 9, DIFFUSION)
    ref = oracle.forward(g, cf, 9)
    assert normrel(gx, ref) <= TOL


def test_recompute_checks_checkpoints_and_matches():
    cf = SETS["AH3"]
    shape = (12, 30, 70)
    x0 = uniform(shape, 300.0, 350.0, 7000)
    p = uniform(shape, 0.0, 1e-3, 7001)
    g = uniform(shape, -1.0, 1.0, 7002)
    a = gpu_adjoint(g, cf, 23, HOTSPOT, tuning={"variant": 2, "k": 3}, recompute=0)
    b = gpu_adjoint(g, cf, 23, HOTSPOT, tuning={"variant": 2, "k": 3}, recompute=1, x0=x0, power=p, ckpt_every=5)
    assert normrel(b[0], a[0]) <= TOL and normrel(b[1], a[1]) <= TOL


def test_run_ckpt_result_and_checkpoints():
    cf = SETS["H2"]
    shape = (90, 310)
    x0 = uniform(shape, 300.0, 350.0, 7100)
    p = uniform(shape, 0.0, 1e-3, 7101)
    plan = S.Plan(HOTSPOT, shape, {"variant": 2, "k": 8})
    try:
        x = dev(x0)
        plan.run_ckpt(x, cf, 29, 7, dev(p))
        torch.cuda.synchronize()
        ref = oracle.forward(x0, cf, 29, power=p, dtype=np.float32)
        assert np.array_equal(x.cpu().numpy(), ref)
    finally:
        plan.close()


def test_autograd_function_against_central_differences():
    """StencilFn gradients vs exact central differences of the quadratic misfit (FP64 oracle)."""
    cf = SETS["AH2"]
    shape = (24, 70)
    T = 9
    x0 = uniform(shape, 300.0, 350.0, 7200)
    p = uniform(shape, 0.0, 1e-3, 7201)
    y = uniform(shape, 300.0, 350.0, 7202)
    xt = dev(x0).requires_grad_(True)
    pt = dev(p).requires_grad_(True)
    out = S.StencilFn.apply(xt, pt, cf, T, 3, 0, {"variant": 2, "k": 4})
    loss = 0.5 * ((out.double() - dev(y).double()) ** 2).sum()
    loss.backward()
    gx = xt.grad.cpu().numpy().astype(np.float64)
    gp = pt.grad.cpu().numpy().astype(np.float64)
    rng = np.random.default_rng(3)
    for _ in range(4):
        idx = tuple(int(rng.integers(0, n)) for n in shape)
        for arr, grad in ((x0, gx), (p, gp)):
            hi = arr.astype(np.float64).copy()
            lo = arr.astype(np.float64).copy()
            hi[idx] += 0.5
            lo[idx] -= 0.5
            args_hi = (hi, p) if arr is x0 else (x0, hi)
            args_lo = (lo, p) if arr is x0 else (x0, lo)
            jp = oracle.loss(oracle.forward(args_hi[0], cf, T, power=args_hi[1]), y)
            jm = oracle.loss(oracle.forward(args_lo[0], cf, T, power=args_lo[1]), y)
            fd = jp - jm
            assert abs(fd - grad[idx]) <= 1e-4 * max(1.0, abs(fd)), (idx, fd, grad[idx])


# ------------------------------------------------------------------ batched

def test_batched_bitwise_equals_oracle_and_replays():
    from workloads import batch_grids
    grids = batch_grids(n2d=6, n3d=3, lo2=20, hi2=300, lo3=5, hi3=40, tlo=1, thi=40, seed=8000)
    xs = [g.field() for g in grids]
    cfs = [SETS[g.coef_set] for g in grids]
    ts = [g.T for g in grids]
    ts[0] = 0
    dts = [dev(x) for x in xs]
    cache = S.run_batched(dts, cfs, ts)
    torch.cuda.synchronize()
    first = [d.cpu().numpy() for d in dts]
    for x, c, T, got in zip(xs, cfs, ts, first):
        ref = oracle.forward(x, c, T, dtype=np.float32)
        assert maxrel(got, ref) <= TOL
        assert np.array_equal(got, ref)
    # replay the captured graph on reset inputs, several times, with eager work in between
    for rep in range(3):
        for d, x in zip(dts, xs):
            d.copy_(dev(x))
        torch.cuda.synchronize()
        S.run_batched(dts, cfs, ts, cache=cache)
        torch.cuda.synchronize()
        for d, f in zip(dts, first):
            assert np.array_equal(d.cpu().numpy(), f), rep
    S.stencil_batch_destroy(cache)


def test_batched_edge_flush_3d_grids():
    """3D grids of the batch at least one window wide and high take the edge-flush tiling in
    the persistent kernel (when every window stays within its neighbours' outputs): results
    must equal the oracle bit for bit, on the first launch and on graph replays."""
    shapes = [(12, 100, 256), (9, 150, 144), (7, 49, 130), (5, 90, 250)]
    xs = [uniform(sh, 0.0, 1.0, 8100 + i) for i, sh in enumerate(shapes)]
    cfs = [SETS["A3"]] * len(shapes)
    ts = [9, 13, 6, 17]
    dts = [dev(x) for x in xs]
    cache = S.run_batched(dts, cfs, ts)
    torch.cuda.synchronize()
    for x, c, T, d in zip(xs, cfs, ts, dts):
        assert np.array_equal(d.cpu().numpy(), oracle.forward(x, c, T, dtype=np.float32)), x.shape
    for rep in range(2):
        for d, x in zip(dts, xs):
            d.copy_(dev(x))
        torch.cuda.synchronize()
        S.run_batched(dts, cfs, ts, cache=cache)
        torch.cuda.synchronize()
        for x, c, T, d in zip(xs, cfs, ts, dts):
            assert np.array_equal(d.cpu().numpy(), oracle.forward(x, c, T, dtype=np.float32)), (rep, x.shape)
    S.stencil_batch_destroy(cache)


def test_t0_is_identity_and_nan_free_small_grids():
    for shape in [(1, 1), (2, 2), (1, 1, 1), (2, 3, 1)]:
        x0 = uniform(shape, 0.0, 1.0, 9)
        check_forward(x0, "A2" if len(shape) == 2 else "A3", 0)
        check_forward(x0, "A2" if len(shape) == 2 else "A3", 7)


# ------------------------------------------------------------------ graph capture

@pytest.mark.parametrize("shape,cset,hot,tuning,T", [
    ((1500, 2060), "AH2", True, {"variant": 2, "k": 8, "seg_len": 8}, 27),   # split 2D pass (two streams)
    ((40, 70, 130), "A3", False, {"variant": 2, "k": 3}, 10),                # balanced 3D launch
])
def test_stencil_run_captured_in_a_graph(shape, cset, hot, tuning, T):
    """stencil_run enqueued on a capturing stream records into a HIP graph (kernels, the
    parity copy, the fork/join of the 2D edge-tile stream); every replay must equal the same
    steps run eagerly, with eager work and synchronisation between the replays."""
    cf = SETS[cset]
    x0 = uniform(shape, 300.0 if hot else 0.0, 350.0 if hot else 1.0, 90)
    p = dev(uniform(shape, 0.0, 1e-3, 91)) if hot else None
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        plan = S.Plan(HOTSPOT if hot else DIFFUSION, shape, tuning)
        ref_plan = S.Plan(HOTSPOT if hot else DIFFUSION, shape, tuning)
    try:
        x = dev(x0)
        y = dev(x0)
        with torch.cuda.stream(s):
            plan.run(x, cf, T, p)  # warm-up outside the capture
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


# ------------------------------------------------------------------ invariants and failure paths

INVARIANT_CASES = [
    ((1500, 2060), "AH2", True, {"variant": 2, "k": 8, "seg_len": 8}),    # split 2D pass
    ((131, 257), "A2", False, {"variant": 2, "k": 12, "seg_len": 40}),    # one 2D launch
    ((40, 70, 130), "AH3", True, {"variant": 2, "k": 3}),                 # balanced 3D launch
    ((33, 50, 129), "A3", False, {"variant": 2, "k": 4, "seg_len": 9}),   # 3D tile launch, odd nx
]


def _inputs(shape, cset, hot, seed):
    x0 = uniform(shape, 300.0 if hot else 0.0, 350.0 if hot else 1.0, seed)
    p = uniform(shape, 0.0, 1e-3, seed + 1) if hot else None
    return SETS[cset], x0, p


@pytest.mark.parametrize("shape,cset,hot,tuning", INVARIANT_CASES)
def test_semigroup_resume_bitwise(shape, cset, hot, tuning):
    """run(T) equals run(t) followed by run(T - t), bit for bit (pass boundaries move)."""
    cf, x0, p = _inputs(shape, cset, hot, 95)
    pw = dev(p) if hot else None
    plan = S.Plan(HOTSPOT if hot else DIFFUSION, shape, tuning)
    try:
        for T, t in ((23, 9), (17, 1), (30, 13)):
            x = dev(x0)
            y = dev(x0)
            plan.run(x, cf, T, pw)
            plan.run(y, cf, t, pw)
            plan.run(y, cf, T - t, pw)
            torch.cuda.synchronize()
            assert torch.equal(x, y), (T, t)
    finally:
        plan.close()


def _guarded(a, guard, fill):
    """A device copy of `a` inside a larger buffer whose guard regions hold `fill`."""
    n = a.size
    buf = torch.full((n + 2 * guard,), fill, dtype=torch.float32, device="cuda")
    view = buf[guard:guard + n].view(a.shape)
    view.copy_(dev(a))
    return buf, view


@pytest.mark.parametrize("shape,cset,hot,tuning", INVARIANT_CASES)
def test_poisoned_scratch_and_guard_canaries(shape, cset, hot, tuning, monkeypatch):
    """With STENCIL_DEBUG_POISON=1 the plan's scratch is NaN before every run, so any read of
    scratch that no pass wrote would poison the result; guard regions around the caller's
    buffers must come back untouched (no stores outside the grid)."""
    monkeypatch.setenv("STENCIL_DEBUG_POISON", "1")
    cf, x0, p = _inputs(shape, cset, hot, 96)
    guard, canary = 4096, 12345.0
    plan = S.Plan(HOTSPOT if hot else DIFFUSION, shape, tuning)
    try:
        for T in (1, 10, 21):
            xb, x = _guarded(x0, guard, canary)
            pb, pw = _guarded(p, guard, canary) if hot else (None, None)
            plan.run(x, cf, T, pw)
            torch.cuda.synchronize()
            ref = oracle.forward(x0, cf, T, power=p, dtype=np.float32)
            assert np.array_equal(x.cpu().numpy(), ref), T
            for b in (xb, pb):
                if b is not None:
                    assert bool(torch.all(b[:guard] == canary)) and bool(torch.all(b[-guard:] == canary)), T
        # the adjoint through guarded outputs
        gb, g = _guarded(uniform(shape, -1.0, 1.0, 97), guard, canary)
        gxb, gx = _guarded(np.zeros(shape, np.float32), guard, canary)
        gpb, gp = _guarded(np.zeros(shape, np.float32), guard, canary) if hot else (None, None)
        plan.adjoint(g, cf, 11, gx, gp)
        torch.cuda.synchronize()
        rx, rp = oracle.adjoint(g.cpu().numpy(), cf, 11, form=HOTSPOT if hot else DIFFUSION)
        assert normrel(gx.cpu().numpy(), rx) <= TOL
        if hot:
            assert normrel(gp.cpu().numpy(), rp) <= TOL
        for b in (gb, gxb, gpb):
            if b is not None:
                assert bool(torch.all(b[:guard] == canary)) and bool(torch.all(b[-guard:] == canary))
    finally:
        plan.close()


def test_injected_fault_is_reported_and_plan_recovers(monkeypatch):
    """A HIP error forced at the second pass (STENCIL_FAULT_INJECT) is returned as
    STENCIL_ERR_HIP through the binding; the same plan then runs correctly."""
    shape, cset = (300, 520), "AH2"
    cf, x0, p = _inputs(shape, cset, True, 98)
    pw = dev(p)
    plan = S.Plan(HOTSPOT, shape, {"variant": 2, "k": 4, "seg_len": 32})
    try:
        x = dev(x0)
        monkeypatch.setenv("STENCIL_FAULT_INJECT", "1")
        with pytest.raises(S.StencilError):
            plan.run(x, cf, 12, pw)
        monkeypatch.delenv("STENCIL_FAULT_INJECT")
        torch.cuda.synchronize()
        x = dev(x0)
        plan.run(x, cf, 12, pw)
        torch.cuda.synchronize()
        assert np.array_equal(x.cpu().numpy(), oracle.forward(x0, cf, 12, power=p, dtype=np.float32))
    finally:
        plan.close()


# ------------------------------------------------------------------ binding argument checks

def test_binding_rejects_tensors_that_do_not_fit_the_plan():
    shape = (40, 64)
    cf = SETS["H2"]
    plan = S.Plan(HOTSPOT, shape, {"variant": 2, "k": 4})
    try:
        good = dev(uniform(shape, 300.0, 350.0, 1))
        pw = dev(uniform(shape, 0.0, 1e-3, 2))
        with pytest.raises(ValueError):  # smaller grid than the plan
            plan.run(dev(uniform((40, 60), 300.0, 350.0, 1)), cf, 3, pw)
        with pytest.raises(ValueError):  # power on the host
            plan.run(good, cf, 3, torch.from_numpy(uniform(shape, 0.0, 1e-3, 2)))
        with pytest.raises(ValueError):  # power of another shape
            plan.run(good, cf, 3, dev(uniform((41, 64), 0.0, 1e-3, 2)))
        with pytest.raises(ValueError):  # hotspot without power
            plan.run(good, cf, 3, None)
        with pytest.raises(ValueError):
            plan.run_ckpt(good, cf, 3, 0, torch.from_numpy(uniform(shape, 0.0, 1e-3, 2)))
        gx = torch.empty_like(good)
        gp_nc = torch.empty((64, 40), device="cuda").t()  # non-contiguous, right shape
        with pytest.raises(ValueError):
            plan.adjoint(good, cf, 3, gx, gp_nc)
        with pytest.raises(ValueError):  # grad_x0 of another shape
            plan.adjoint(good, cf, 3, torch.empty((40, 63), device="cuda"))
        # the plan still works after the rejections
        plan.run(good, cf, 3, pw)
        torch.cuda.synchronize()
    finally:
        plan.close()


def test_grad_power_offset_by_four_bytes():
    """grad_p that is only 4-byte aligned takes the scalar path and matches the aligned one."""
    shape = (33, 256)
    cf = SETS["AH2"]
    g = dev(uniform(shape, -1.0, 1.0, 77))
    plan = S.Plan(HOTSPOT, shape, {"variant": 2, "k": 4})
    try:
        gx = torch.empty_like(g)
        gp = torch.empty_like(g)
        plan.adjoint(g, cf, 9, gx, gp)
        big = torch.empty(g.numel() + 1, device="cuda")
        gp_off = big[1:].view(shape)  # contiguous, 4 bytes past a 16-byte boundary
        gx2 = torch.empty_like(g)
        plan.adjoint(g, cf, 9, gx2, gp_off)
        torch.cuda.synchronize()
        assert np.array_equal(gp.cpu().numpy(), gp_off.cpu().numpy())
        assert np.array_equal(gx.cpu().numpy(), gx2.cpu().numpy())
    finally:
        plan.close()
    rx, rp = oracle.adjoint(g.cpu().numpy(), cf, 9, form=HOTSPOT)
    assert normrel(gp.cpu().numpy(), rp) <= TOL


def test_autograd_retain_graph_and_plan_reuse():
    """backward twice on one graph (retain_graph) gives the same gradients; a later forward of
    the same shape reuses the released plan."""
    cf = SETS["AH2"]
    shape = (20, 50)
    x0 = uniform(shape, 300.0, 350.0, 7300)
    p = uniform(shape, 0.0, 1e-3, 7301)
    xt = dev(x0).requires_grad_(True)
    pt = dev(p).requires_grad_(True)
    out = S.StencilFn.apply(xt, pt, cf, 7, 3, 0, {"variant": 2, "k": 4})
    loss = (out.double() ** 2).sum()
    loss.backward(retain_graph=True)
    g1 = (xt.grad.clone(), pt.grad.clone())
    xt.grad = None
    pt.grad = None
    loss.backward()
    assert torch.equal(g1[0], xt.grad) and torch.equal(g1[1], pt.grad)
    del out, loss
    out2 = S.StencilFn.apply(xt, pt, cf, 7, 3, 0, {"variant": 2, "k": 4})
    assert np.array_equal(out2.detach().cpu().numpy(), oracle.forward(x0, cf, 7, power=p, dtype=np.float32))
