"""Grids beyond 2^31 cells: every index of the path is 64-bit where it must be.

The fields are integer patterns formed on the device (no host copy of a 10 GB array); the
oracle runs on the sub-grid within T cells of each sampled output (the cone that determines
it, cut at the real grid edges), built from the same pattern, so its value is expected bit for
bit.  Samples include cells whose flat index exceeds 2^31.
"""
import numpy as np
import pytest

import oracle
import paper_1802_00438_amd as S
from workloads import SETS, STAR_SETS, HOTSPOT, DIFFUSION

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def pattern_np(idx_arrays, mult, mod, scale, offset):
    acc = np.zeros(np.broadcast(*idx_arrays).shape, dtype=np.int64)
    for a, m in zip(idx_arrays, mult):
        acc = acc + a.astype(np.int64) * m
    return (offset + (acc % mod).astype(np.float32) * np.float32(scale)).astype(np.float32)


def pattern_dev(shape, mult, mod, scale, offset):
    out = torch.zeros(shape, dtype=torch.int32, device="cuda")
    for ax, (n, m) in enumerate(zip(shape, mult)):
        view = [1] * len(shape)
        view[ax] = n
        out += (torch.arange(n, dtype=torch.int32, device="cuda") * m).view(view)
    out.remainder_(mod)
    f = out.to(torch.float32)
    del out
    f.mul_(np.float32(scale)).add_(np.float32(offset))
    return f


def cone(shape, idx, T, mult, mod, scale, offset):
    sl = [slice(max(0, i - T), min(n, i + T + 1)) for i, n in zip(idx, shape)]
    grids = np.meshgrid(*[np.arange(s.start, s.stop) for s in sl], indexing="ij")
    return pattern_np(grids, mult, mod, scale, offset), tuple(i - s.start for i, s in zip(idx, sl))


def flat(idx, shape):
    f = 0
    for i, n in zip(idx, shape):
        f = f * n + i
    return f


def test_hotspot2d_beyond_2_31_cells():
    shape = (40000, 65536)  # 2.62e9 cells, 10.5 GB per field
    T = 24
    fx = ((131, 17), 997, 50.0 / 997, 300.0)
    fp = ((7, 29), 1009, 1e-3 / 1009, 0.0)
    x = pattern_dev(shape, *fx)
    p = pattern_dev(shape, *fp)
    plan = S.Plan(HOTSPOT, shape, {"variant": 2, "k": 12, "seg_len": 192})
    try:
        plan.run(x, SETS["H2"], T, p)
        torch.cuda.synchronize()
    finally:
        plan.close()
    samples = [(0, 0), (39999, 65535), (33000, 1234), (20000, 65535), (39999, 0), (17, 40000)]
    assert max(flat(i, shape) for i in samples) > 2 ** 31
    for idx in samples:
        xs, loc = cone(shape, idx, T, *fx)
        ps, _ = cone(shape, idx, T, *fp)
        ref = oracle.forward(xs, SETS["H2"], T, power=ps, dtype=np.float32)[loc]
        got = x[idx].item()
        assert got == ref, (idx, got, ref)


def test_diffusion3d_beyond_2_31_cells():
    shape = (1300, 1300, 1300)  # 2.2e9 cells, 8.8 GB
    T = 8
    fx = ((7, 131, 17), 997, 1.0 / 997, 0.0)
    x = pattern_dev(shape, *fx)
    plan = S.Plan(DIFFUSION, shape, {"variant": 2, "k": 4})
    try:
        plan.run(x, SETS["D3"], T)
        torch.cuda.synchronize()
    finally:
        plan.close()
    samples = [(0, 0, 0), (1299, 1299, 1299), (1290, 5, 700), (700, 1299, 3)]
    assert max(flat(i, shape) for i in samples) > 2 ** 31
    for idx in samples:
        xs, loc = cone(shape, idx, T, *fx)
        ref = oracle.forward(xs, SETS["D3"], T, dtype=np.float32)[loc]
        got = x[idx].item()
        assert got == ref, (idx, got, ref)


def test_star2d_beyond_2_31_cells():
    shape = (40000, 65536)
    r, T = 2, 8
    fx = ((131, 17), 997, 1.0 / 997, 0.0)
    x = pattern_dev(shape, *fx)
    plan = S.StarPlan(r, shape, {"variant": 2, "k": 4, "seg_len": 192})
    try:
        plan.run(x, STAR_SETS[r], T)
        torch.cuda.synchronize()
    finally:
        plan.close()
    for idx in [(0, 0), (39999, 65535), (33000, 1234), (39998, 65534)]:
        xs, loc = cone(shape, idx, r * T, *fx)
        ref = oracle.star2d(xs, STAR_SETS[r], T, dtype=np.float32)[loc]
        got = x[idx].item()
        assert got == ref, (idx, got, ref)
