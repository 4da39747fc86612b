"""Full-size parity at the shapes and launch configuration the bench times.

A cell's value after T steps depends only on the initial cells within T steps of it (the
stencil has radius 1), so the oracle can reproduce sampled output cells exactly by running
on the sub-grid of cells within distance T, cut at the real grid edges: the artificial edges
of the sub-grid need T steps to reach the sampled cell.  The FP32 oracle then performs the
very same operations for that cell as on the full grid, so the GPU value is expected bit for
bit (and is required within max-rel 1e-5).

For the 3D hotspot adjoint problem the operator is symmetric (mirror-symmetric weights), so
the oracle's forward pass gives the exact full-size references: grad_x0 = A^T g (linear part
of the forward map applied to the cotangent), and grad_p = cp * sum_{j<T} A^j g, which is the
hotspot forward map started from zero with the cotangent as its power map and no ambient term.
"""
import numpy as np
import pytest

import oracle
import paper_1802_00438_amd as S
from workloads import WORKLOADS, SETS, DIFFUSION, HOTSPOT, HOTSPOT_PHYS

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL = 1e-5


def cone_sample(x0, power, cf, T, idx, dtype=np.float32, form=None):
    """Oracle value of output cell idx after T steps, from the sub-grid of radius T."""
    sl = tuple(slice(max(0, i - T), min(n, i + T + 1)) for i, n in zip(idx, x0.shape))
    sub = np.ascontiguousarray(x0[sl])
    psub = np.ascontiguousarray(power[sl]) if power is not None else None
    out = oracle.forward(sub, cf, T, power=psub, dtype=dtype, form=form)
    return out[tuple(i - s.start for i, s in zip(idx, sl))]


def test_hotspot2d_16384_full_size_samples():
    wl = WORKLOADS["hotspot2d_16384"]
    x0 = wl.field()
    p = wl.power()
    x = torch.from_numpy(x0).cuda()
    pw = torch.from_numpy(p).cuda()
    plan = S.Plan(HOTSPOT, wl.shape)  # auto-tuned, as the bench runs it
    try:
        plan.run(x, wl.coeffs, wl.T, pw)
        torch.cuda.synchronize()
        got = x.cpu().numpy()
    finally:
        plan.close()
    assert np.isfinite(got).all()
    n = wl.nx
    for idx in [(n // 2 + 17, n // 3 + 5), (0, 0), (n - 1, 12345), (777, n - 1), (n - 1, n - 1)]:
        ref = cone_sample(x0, p, wl.coeffs, wl.T, idx)
        g = got[idx]
        assert abs(g - ref) / abs(ref) <= TOL, (idx, g, ref)
        assert g == ref, (idx, g, ref)
    # a property that holds at any size: the field stays within the bounds of the fixed point
    # and the initial data (convex weights plus a non-negative source)
    assert got.min() >= 80.0 and got.max() <= 350.0 + wl.T * 64 * 1e-3 + 1.0


def test_hotspot2d_phys_16384_full_size_samples():
    """The physical-form workload at its full size, auto-tuned as the bench runs it."""
    wl = WORKLOADS["hotspot2d_phys_16384"]
    x0 = wl.field()
    p = wl.power()
    x = torch.from_numpy(x0).cuda()
    pw = torch.from_numpy(p).cuda()
    plan = S.Plan(HOTSPOT_PHYS, wl.shape)
    try:
        plan.run(x, wl.coeffs, wl.T, pw)
        torch.cuda.synchronize()
        got = x.cpu().numpy()
    finally:
        plan.close()
    assert np.isfinite(got).all()
    n = wl.nx
    for idx in [(n // 2 + 3, n // 5 + 11), (0, 0), (n - 1, 4321), (1234, n - 1)]:
        ref = cone_sample(x0, p, wl.coeffs, wl.T, idx, form=HOTSPOT_PHYS)
        g = got[idx]
        assert abs(g - ref) / abs(ref) <= TOL, (idx, g, ref)
        assert g == ref, (idx, g, ref)
    assert got.min() >= 80.0 and got.max() <= 350.0 + wl.T * 64 * 1e-3 + 1.0


def test_diffusion3d_512_full_size_samples():
    wl = WORKLOADS["diffusion3d_512"]
    x0 = wl.field()
    x = torch.from_numpy(x0).cuda()
    samples = [(0, 0, 0), (511, 300, 7), (100, 511, 256)]
    refs = [cone_sample(x0, None, wl.coeffs, wl.T, idx) for idx in samples]
    for tuning in (None, {"variant": 1}):
        xx = x.clone()
        plan = S.Plan(DIFFUSION, wl.shape, tuning)
        try:
            plan.run(xx, wl.coeffs, wl.T)
            torch.cuda.synchronize()
            got = xx.cpu().numpy()
        finally:
            plan.close()
        for idx, ref in zip(samples, refs):
            assert abs(got[idx] - ref) / abs(ref) <= TOL, (tuning, idx, got[idx], ref)
            assert got[idx] == ref, (tuning, idx, got[idx], ref)
        # maximum principle (convex weights)
        assert got.min() >= x0.min() - 1e-6 and got.max() <= x0.max() + 1e-6


def test_hotspot3d_256_adjoint_full_size():
    wl = WORKLOADS["hotspot3d_256_adjoint"]
    cf = wl.coeffs
    x0 = wl.field()
    p = wl.power()
    y = wl.target()
    plan = S.Plan(HOTSPOT, wl.shape)
    try:
        x = torch.from_numpy(x0).cuda()
        pw = torch.from_numpy(p).cuda()
        plan.run_ckpt(x, cf, wl.T, wl.ckpt_every, pw)
        g = (x - torch.from_numpy(y).cuda()).contiguous()
        gx = torch.empty_like(g)
        gp = torch.empty_like(g)
        plan.adjoint(g, cf, wl.T, gx, gp, pw, 1)  # recompute=1 checks every checkpoint bitwise
        torch.cuda.synchronize()
        gh, gxh, gph = g.cpu().numpy(), gx.cpu().numpy(), gp.cpu().numpy()
    finally:
        plan.close()
    lin = cf.copy()
    lin[7:] = 0.0
    ref_x = oracle.forward(gh, lin, wl.T, form=DIFFUSION, dtype=np.float32)
    src = cf.copy()
    src[8] = 0.0  # no ambient term: the source is cp * g
    ref_p = oracle.forward(np.zeros_like(gh), src, wl.T, power=gh, form=HOTSPOT, dtype=np.float32)
    # The cotangent x_T - y keeps one sign (x_T stays below the target's range), and the
    # weights are non-negative, so no gradient entry comes near zero: the comparison is
    # element by element.
    assert np.all(gh < 0)
    for got, ref in ((gxh, ref_x), (gph, ref_p)):
        rel = np.abs(got.astype(np.float64) - ref) / np.abs(ref.astype(np.float64))
        assert float(rel.max()) <= TOL, float(rel.max())
