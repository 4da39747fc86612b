"""GPU parity over a seeded random sweep of shapes, step counts and blockings.

The hand-picked shapes of the other parity tests aim at known corner cases (one tile, a tail
of one cell, windows flush with an edge).  Here every case draws its grid size log-uniformly,
its step count, fused-step count and segment length uniformly, and its form and coefficient
set from the library's whole surface (2D diffusion, Rodinia hotspot and Table 2's physical
hotspot; 3D diffusion and hotspot with the tile and the balanced launch; radius-r stars in 2D
and 3D, in both forms, and their adjoint), so
that tilings nobody thought of get exercised too.  The bar is the same: bit-identical to the
FP32 oracle (each kernel keeps the oracle's FMA order), and within max-rel 1e-5 of it.
"""
import math

import numpy as np
import pytest

import oracle
import paper_1802_00438_amd as S
from workloads import SETS, STAR_SETS, STAR3_SETS, DIFFUSION, HOTSPOT, HOTSPOT_PHYS, rng, uniform

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL = 1e-5
N2D, N3D, NSTAR = 96, 64, 48

# largest fused-step count served per (dimensionality, form); any k up to it runs on the
# smallest instantiated kernel at or above it
KMAX_2D = {DIFFUSION: 24, HOTSPOT: 16, HOTSPOT_PHYS: 16}
KMAX_3D = {DIFFUSION: 6, HOTSPOT: 4}
KMAX_STAR = {1: 8, 2: 8, 3: 4, 4: 4}


def log_uniform(g, lo, hi):
    return int(round(math.exp(g.uniform(math.log(lo), math.log(hi)))))


def maxrel(a, b):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    return float(np.max(np.abs(a - b) / np.maximum(np.abs(b), 1e-30))) if a.size else 0.0


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()


def draw_2d(i):
    g = rng(9100 + i)
    form = [DIFFUSION, HOTSPOT, HOTSPOT_PHYS][i % 3]
    cset = {DIFFUSION: ["D2", "A2"], HOTSPOT: ["H2", "AH2"], HOTSPOT_PHYS: ["HP2", "HPr"]}[form][int(g.integers(2))]
    lo = 1 if i % 4 == 0 else 150  # every fourth case small, the rest several tiles wide
    shape = (log_uniform(g, lo, 2000), log_uniform(g, lo, 2000))
    T = int(g.integers(0, 61))
    k = int(g.integers(1, KMAX_2D[form] + 1))
    seg = int(g.integers(1, 400))
    return form, cset, shape, T, {"variant": 2, "k": k, "seg_len": seg}


def draw_3d(i):
    g = rng(9200 + i)
    form = [DIFFUSION, HOTSPOT][i % 2]
    cset = {DIFFUSION: ["D3", "A3"], HOTSPOT: ["H3", "AH3", "H3p"]}[form][int(g.integers(2 if form == DIFFUSION else 3))]
    lo = 1 if i % 4 == 3 else 24
    shape = (log_uniform(g, 1, 80), log_uniform(g, lo, 200), log_uniform(g, 2 * lo, 400))
    T = int(g.integers(0, 15))
    k = int(g.integers(1, KMAX_3D[form] + 1))
    # segment length 0 with k given: the balanced launch; otherwise one workgroup per tile
    seg = 0 if (i // 2) % 2 == 0 else int(g.integers(1, 80))
    return form, cset, shape, T, {"variant": 2, "k": k, "seg_len": seg}


def draw_star(i):
    g = rng(9300 + i)
    r = 1 + i % 4
    lo = 1 if i % 4 == 0 else 100
    shape = (log_uniform(g, lo, 1500), log_uniform(g, lo, 1500))
    T = int(g.integers(0, 31))
    k = int(g.integers(1, KMAX_STAR[r] + 1))
    seg = int(g.integers(1, 300))
    return r, shape, T, {"variant": 2, "k": k, "seg_len": seg}


def fields(form, shape, seed):
    if form == DIFFUSION:
        return uniform(shape, 0.0, 1.0, seed), None
    return uniform(shape, 300.0, 350.0, seed), uniform(shape, 0.0, 1e-3, seed + 1)


def run_and_compare(form, cset, shape, T, tuning, seed):
    cf = SETS[cset]
    x0, p = fields(form, shape, seed)
    x = dev(x0)
    plan = S.Plan(form, shape, tuning)
    try:
        plan.run(x, cf, T, dev(p) if p is not None else None)
        torch.cuda.synchronize()
        used = plan.tuning
    finally:
        plan.close()
    got = x.cpu().numpy()
    ref = oracle.forward(x0, cf, T, power=p, form=form, dtype=np.float32)
    case = (form, cset, shape, T, tuning, used)
    assert maxrel(got, ref) <= TOL, case
    assert np.array_equal(got, ref), (case, maxrel(got, ref))


@pytest.mark.parametrize("i", range(N2D))
def test_random_2d(i):
    form, cset, shape, T, tuning = draw_2d(i)
    print("case 2d", i, form, cset, shape, T, tuning, flush=True)
    run_and_compare(form, cset, shape, T, tuning, 9500 + i)


@pytest.mark.parametrize("i", range(N3D))
def test_random_3d(i):
    form, cset, shape, T, tuning = draw_3d(i)
    print("case 3d", i, form, cset, shape, T, tuning, flush=True)
    run_and_compare(form, cset, shape, T, tuning, 9600 + i)


@pytest.mark.parametrize("i", range(NSTAR))
def test_random_star(i):
    r, shape, T, tuning = draw_star(i)
    print("case star", i, r, shape, T, tuning, flush=True)
    if r == 1:
        cf = SETS["A2"]  # cc, cw, ce, cn, cs -> cc, w1, e1, s1, n1
        w = np.array([cf[0], cf[1], cf[2], cf[4], cf[3]], dtype=np.float32)
    else:
        w = STAR_SETS[r]
    x0 = uniform(shape, 0.0, 1.0, 9700 + i)
    x = dev(x0)
    plan = S.StarPlan(r, shape, tuning)
    try:
        plan.run(x, w, T)
        torch.cuda.synchronize()
        used = plan.tuning
    finally:
        plan.close()
    got = x.cpu().numpy()
    ref = oracle.star2d(x0, w, T, dtype=np.float32)
    assert maxrel(got, ref) <= TOL, (r, shape, T, tuning, used)
    assert np.array_equal(got, ref), (r, shape, T, tuning, used, maxrel(got, ref))


# ------------------------------------------------------------------ radius-r 3D, hotspot form, adjoint

NSTAR3, NSTARADJ = 40, 32
KMAX_STAR3 = {1: 3, 2: 2, 3: 2, 4: 1}
STAR_SRC = (0.125, 2.0 ** -8, 80.0)  # cp, c_amb, t_amb of the hotspot form


def star_w(r, ndim, scale=1.0):
    if ndim == 3:
        w = STAR3_SETS[r]
    elif r == 1:
        cf = SETS["A2"]
        w = np.array([cf[0], cf[1], cf[2], cf[4], cf[3]], dtype=np.float32)
    else:
        w = STAR_SETS[r]
    return (w.astype(np.float64) * scale).astype(np.float32)


def draw_star3(i):
    g = rng(9350 + i)
    r = 1 + i % 4
    lo = 1 if i % 4 == 2 else 20
    shape = (log_uniform(g, 1, 60), log_uniform(g, lo, 200), log_uniform(g, lo, 300))
    T = int(g.integers(0, 16))
    k = int(g.integers(1, KMAX_STAR3[r] + 1))
    seg = int(g.integers(1, 80))
    return r, shape, T, {"variant": 2, "k": k, "seg_len": seg}, bool(i % 2)


@pytest.mark.parametrize("i", range(NSTAR3))
def test_random_star3d(i):
    """3D radius-r stars, half of them in the hotspot form, bit for bit against the oracle."""
    r, shape, T, tuning, hot = draw_star3(i)
    print("case star3d", i, r, shape, T, tuning, hot, flush=True)
    w = star_w(r, 3, 0.875 if hot else 1.0)
    x0 = uniform(shape, 300.0, 350.0, 9750 + i) if hot else uniform(shape, 0.0, 1.0, 9750 + i)
    p = uniform(shape, 0.0, 1.0, 9790 + i) if hot else None
    x = dev(x0)
    plan = S.StarPlan(r, shape, tuning)
    try:
        if hot:
            plan.run(x, w, T, power=dev(p), src=STAR_SRC)
        else:
            plan.run(x, w, T)
        torch.cuda.synchronize()
        used = plan.tuning
    finally:
        plan.close()
    got = x.cpu().numpy()
    ref = oracle.star3d(x0, w, T, dtype=np.float32, power=p, src=STAR_SRC if hot else None)
    assert np.array_equal(got, ref), (r, shape, T, tuning, hot, used, maxrel(got, ref))


@pytest.mark.parametrize("i", range(NSTAR // 2))
def test_random_star2d_hotspot(i):
    """The draws of the 2D star sweep in the hotspot form."""
    r, shape, T, tuning = draw_star(i)
    print("case star2d hot", i, r, shape, T, tuning, flush=True)
    w = star_w(r, 2, 0.875)
    x0 = uniform(shape, 300.0, 350.0, 9800 + i)
    p = uniform(shape, 0.0, 1.0, 9840 + i)
    x = dev(x0)
    plan = S.StarPlan(r, shape, tuning)
    try:
        plan.run(x, w, T, power=dev(p), src=STAR_SRC)
        torch.cuda.synchronize()
    finally:
        plan.close()
    got = x.cpu().numpy()
    ref = oracle.star2d(x0, w, T, dtype=np.float32, power=p, src=STAR_SRC)
    assert np.array_equal(got, ref), (r, shape, T, tuning, maxrel(got, ref))


def draw_star_adj(i):
    g = rng(9400 + i)
    r = 1 + i % 4
    if i % 2:
        shape = (log_uniform(g, 1, 40), log_uniform(g, 1, 120), log_uniform(g, 1, 300))
    else:
        shape = (log_uniform(g, 1, 600), log_uniform(g, 1, 600))
    if i % 3 == 0:  # rows of whole 16-byte groups: the four-cells-per-lane kernel
        shape = shape[:-1] + (4 * max(1, shape[-1] // 4),)
    T = int(g.integers(0, 13))
    return r, shape, T, bool(i % 4 >= 2)


@pytest.mark.parametrize("i", range(NSTARADJ))
def test_random_star_adjoint(i):
    """The radius-r adjoint within 1e-5 elementwise of the FP64 oracle (positive cotangents)."""
    r, shape, T, hot = draw_star_adj(i)
    print("case star adjoint", i, r, shape, T, hot, flush=True)
    w = star_w(r, len(shape))
    lam = uniform(shape, 0.5, 1.5, 9900 + i)
    plan = S.StarPlan(r, shape, {"variant": 2, "k": 1})
    try:
        gx = torch.empty(shape, device="cuda")
        gp = torch.empty(shape, device="cuda") if hot else None
        plan.adjoint(dev(lam), w, T, gx, gp, STAR_SRC if hot else None)
        torch.cuda.synchronize()
    finally:
        plan.close()
    ref, refp = oracle.star_adjoint(lam, w, T, cp=STAR_SRC[0] if hot else None)
    assert maxrel(gx.cpu().numpy(), ref) <= TOL, (r, shape, T, hot)
    if hot and T > 0:
        assert maxrel(gp.cpu().numpy(), refp) <= TOL, (r, shape, T)


def test_draws_cover_the_surface():
    """The sweep reaches every form, both 3D launch shapes, every radius and odd sizes."""
    d2 = [draw_2d(i) for i in range(N2D)]
    d3 = [draw_3d(i) for i in range(N3D)]
    ds = [draw_star(i) for i in range(NSTAR)]
    assert {f for f, *_ in d2} == {DIFFUSION, HOTSPOT, HOTSPOT_PHYS}
    assert {t["seg_len"] == 0 for *_, t in d3} == {True, False}
    assert {r for r, *_ in ds} == {1, 2, 3, 4}
    assert any(s[0] % 2 for _, _, s, _, _ in d2) and any(s[2] % 2 for _, _, s, _, _ in d3)
    d3s = [draw_star3(i) for i in range(NSTAR3)]
    assert {r for r, *_ in d3s} == {1, 2, 3, 4} and {h for *_, h in d3s} == {True, False}
    da = [draw_star_adj(i) for i in range(NSTARADJ)]
    assert {len(s) for _, s, _, _ in da} == {2, 3} and {h for *_, h in da} == {True, False}
    assert any(s[-1] % 4 == 0 for _, s, _, _ in da) and any(s[-1] % 4 for _, s, _, _ in da)


# ------------------------------------------------------------------ adjoint sweep

NADJ = 48
KMAX_ADJ = {2: 12, 3: 4}


def draw_adjoint(i):
    g = rng(9400 + i)
    ndim = 2 if i % 3 else 3
    if ndim == 2:
        form = [DIFFUSION, HOTSPOT, HOTSPOT_PHYS][(i // 3) % 3]
        cset = {DIFFUSION: "A2", HOTSPOT: "AH2", HOTSPOT_PHYS: "HPr"}[form]
        lo = 1 if i % 5 == 0 else 100
        shape = (log_uniform(g, lo, 1200), log_uniform(g, lo, 1200))
        T = int(g.integers(0, 31))
    else:
        form = [DIFFUSION, HOTSPOT][(i // 3) % 2]
        cset = {DIFFUSION: "A3", HOTSPOT: "AH3"}[form]
        lo = 1 if i % 5 == 0 else 24
        shape = (log_uniform(g, 1, 60), log_uniform(g, lo, 150), log_uniform(g, 2 * lo, 300))
        T = int(g.integers(0, 13))
    k = int(g.integers(1, KMAX_ADJ[ndim] + 1))
    seg = int(g.integers(1, 200))
    # every fourth case recomputes the forward tiles from checkpoints (and verifies them)
    recompute = 1 if (i % 4 == 1 and T > 0) else 0
    ckpt_every = int(g.integers(1, T + 1)) if recompute else 0
    return form, cset, shape, T, {"variant": 2, "k": k, "seg_len": seg}, recompute, ckpt_every


@pytest.mark.parametrize("i", range(NADJ))
def test_random_adjoint(i):
    form, cset, shape, T, tuning, recompute, ckpt_every = draw_adjoint(i)
    print("case adjoint", i, form, cset, shape, T, tuning, recompute, ckpt_every, flush=True)
    cf = SETS[cset]
    cot = uniform(shape, -1.0, 1.0, 9800 + i)
    x0, p = fields(form, shape, 9900 + i)
    hot = form != DIFFUSION
    plan = S.Plan(form, shape, tuning)
    try:
        c = dev(cot)
        gx = torch.empty_like(c)
        gp = torch.empty_like(c) if hot else None
        pw = dev(p) if hot else None
        if recompute:
            plan.run_ckpt(dev(x0), cf, T, ckpt_every, pw)
        plan.adjoint(c, cf, T, gx, gp, pw, recompute)
        torch.cuda.synchronize()
    finally:
        plan.close()
    rx, rp = oracle.adjoint(cot, cf, T, form=form)
    gxn = gx.cpu().numpy()
    scale = max(float(np.max(np.abs(rx))), 1e-300)
    assert float(np.max(np.abs(gxn - rx))) / scale <= TOL, (form, cset, shape, T, tuning)
    if hot:
        gpn = gp.cpu().numpy()
        scale = max(float(np.max(np.abs(rp))), 1e-300)
        assert float(np.max(np.abs(gpn - rp))) / scale <= TOL, (form, cset, shape, T, tuning)


def test_adjoint_draws_cover_the_surface():
    d = [draw_adjoint(i) for i in range(NADJ)]
    assert {(len(s), f) for f, _, s, *_ in d} == {(2, DIFFUSION), (2, HOTSPOT), (2, HOTSPOT_PHYS), (3, DIFFUSION),
                                                 (3, HOTSPOT)}
    assert any(r for *_, r, _ in d) and any(T == 0 for _, _, _, T, *_ in d)


# ------------------------------------------------------------------ batched sweep

NBATCH = 8


def draw_batch(b):
    """A batch of 2-12 diffusion grids of mixed dimensionality, sizes and step counts."""
    g = rng(9450 + b)
    n = int(g.integers(2, 13))
    out = []
    for j in range(n):
        lo = 1 if j % 2 else 40  # half the grids small, half several windows wide
        if g.random() < 0.6:
            shape = (log_uniform(g, lo, 700), log_uniform(g, 3 * lo, 900))
            cset = ["D2", "A2"][int(g.integers(2))]
        else:
            shape = (log_uniform(g, 1, 48), log_uniform(g, lo, 160), log_uniform(g, 3 * lo, 300))
            cset = ["D3", "A3"][int(g.integers(2))]
        out.append((shape, cset, int(g.integers(0, 45))))
    return out


@pytest.mark.parametrize("b", range(NBATCH))
def test_random_batched(b):
    batch = draw_batch(b)
    print("case batch", b, batch, flush=True)
    xs = [uniform(sh, 0.0, 1.0, 10000 + 100 * b + j) for j, (sh, _, _) in enumerate(batch)]
    cfs = [SETS[c] for _, c, _ in batch]
    ts = [T for _, _, T in batch]
    dts = [dev(x) for x in xs]
    refs = [oracle.forward(x, c, T, dtype=np.float32) for x, c, T in zip(xs, cfs, ts)]
    cache = S.run_batched(dts, cfs, ts)
    try:
        torch.cuda.synchronize()
        for (sh, c, T), d, ref in zip(batch, dts, refs):
            assert np.array_equal(d.cpu().numpy(), ref), (sh, c, T)
        # one graph replay on reset inputs
        for d, x in zip(dts, xs):
            d.copy_(dev(x))
        torch.cuda.synchronize()
        S.run_batched(dts, cfs, ts, cache=cache)
        torch.cuda.synchronize()
        for (sh, c, T), d, ref in zip(batch, dts, refs):
            assert np.array_equal(d.cpu().numpy(), ref), ("replay", sh, c, T)
    finally:
        S.stencil_batch_destroy(cache)


# ------------------------------------------------------------------ checkpointed forward sweep

NCKPT = 24


@pytest.mark.parametrize("i", range(NCKPT))
def test_random_checkpointed_forward(i):
    """run_ckpt with a random checkpoint interval (0: the library's sqrt(T)) ends on the same
    field as the oracle, bit for bit, whatever the interval and the blocking."""
    form, cset, shape, T, tuning = draw_2d(i) if i % 2 == 0 else draw_3d(i)
    g = rng(9470 + i)
    every = 0 if i % 3 == 0 else int(g.integers(1, max(T, 1) + 1))
    print("case ckpt", i, form, cset, shape, T, tuning, every, flush=True)
    cf = SETS[cset]
    x0, p = fields(form, shape, 10900 + i)
    x = dev(x0)
    plan = S.Plan(form, shape, tuning)
    try:
        plan.run_ckpt(x, cf, T, every, dev(p) if p is not None else None)
        torch.cuda.synchronize()
    finally:
        plan.close()
    ref = oracle.forward(x0, cf, T, power=p, form=form, dtype=np.float32)
    assert np.array_equal(x.cpu().numpy(), ref), (form, cset, shape, T, tuning, every)
