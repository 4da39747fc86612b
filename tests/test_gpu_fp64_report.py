"""FP32 GPU results against the FP64 oracle, per workload, at the workloads' real sizes.

The parity bar is the FP32 oracle (max-rel 1e-5; the kernels are in fact bit-identical to
it).  These tests report how far the FP32 result is from the FP64 oracle for every workload
and check a loose bound from FP32 rounding: one step rounds each cell a few times relative to
its magnitude, and the weights are convex, so the relative error grows at most linearly with
T: max-rel <= 8 * T * 2^-24.

Large grids are sampled with the radius-T cone: the oracle runs on the sub-grid of cells
within T steps of the sampled cell (cut at the real grid edges), whose artificial edges need
T steps to reach it, so the FP64 value of that cell equals the full grid's.
"""
import numpy as np
import pytest

import oracle
import paper_1802_00438_amd as S
from conftest import FP64_REPORT
from workloads import WORKLOADS, SETS, DIFFUSION, HOTSPOT, STAR_SETS, STAR_WORKLOAD, batch_grids, star_field

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def maxrel(a, b):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    return float(np.max(np.abs(a - b) / np.maximum(np.abs(b), 1e-30)))


def bound(T):
    return 8.0 * max(T, 1) * 2.0 ** -24


def cone64(x0, power, cf, T, idx, form=None):
    sl = tuple(slice(max(0, i - T), min(n, i + T + 1)) for i, n in zip(idx, x0.shape))
    sub = np.ascontiguousarray(x0[sl])
    psub = np.ascontiguousarray(power[sl]) if power is not None else None
    out = oracle.forward(sub, cf, T, power=psub, dtype=np.float64, form=form)
    return out[tuple(i - s.start for i, s in zip(idx, sl))]


def gpu_run(wl, x0, power):
    x = torch.from_numpy(x0).cuda()
    p = torch.from_numpy(power).cuda() if power is not None else None
    plan = S.Plan(wl.form, wl.shape)
    try:
        plan.run(x, wl.coeffs, wl.T, p)
        torch.cuda.synchronize()
    finally:
        plan.close()
    return x.cpu().numpy()


def report(name, what, err, note, T):
    FP64_REPORT.append((name, what, err, note))
    assert err <= bound(T), (name, what, err, bound(T))


def test_fp64_diffusion2d_256():
    wl = WORKLOADS["diffusion2d_256"]
    x0 = wl.field()
    got = gpu_run(wl, x0, None)
    ref = oracle.forward(x0, wl.coeffs, wl.T, dtype=np.float64)
    report(wl.name, "forward, all cells", maxrel(got, ref), "T=%d" % wl.T, wl.T)


def test_fp64_hotspot2d_16384():
    wl = WORKLOADS["hotspot2d_16384"]
    x0, p = wl.field(), wl.power()
    got = gpu_run(wl, x0, p)
    n = wl.nx
    idx = [(n // 2 + 17, n // 3 + 5), (0, 0), (n - 1, 12345)]
    err = max(abs(float(got[i]) - cone64(x0, p, wl.coeffs, wl.T, i)) / abs(cone64(x0, p, wl.coeffs, wl.T, i))
              for i in idx)
    report(wl.name, "forward, %d cone samples" % len(idx), err, "T=%d" % wl.T, wl.T)


def test_fp64_hotspot2d_phys_16384():
    wl = WORKLOADS["hotspot2d_phys_16384"]
    x0, p = wl.field(), wl.power()
    got = gpu_run(wl, x0, p)
    n = wl.nx
    idx = [(n // 2 + 3, n // 5 + 11), (0, 0), (n - 1, 4321)]
    refs = [cone64(x0, p, wl.coeffs, wl.T, i, form=wl.form) for i in idx]
    err = max(abs(float(got[i]) - r) / abs(r) for i, r in zip(idx, refs))
    report(wl.name, "forward, %d cone samples" % len(idx), err, "T=%d" % wl.T, wl.T)


def test_fp64_star2d_r2_16384():
    wl = STAR_WORKLOAD
    r, T = wl["rad"], wl["T"]
    x0 = star_field(wl)
    x = torch.from_numpy(x0).cuda()
    plan = S.StarPlan(r, x0.shape)
    try:
        plan.run(x, STAR_SETS[r], T)
        torch.cuda.synchronize()
    finally:
        plan.close()
    got = x.cpu().numpy()
    n = wl["nx"]
    errs = []
    for idx in [(n // 2 + 7, n // 3 + 1), (0, 0)]:
        sl = tuple(slice(max(0, i - r * T), min(n, i + r * T + 1)) for i in idx)
        ref = oracle.star2d(np.ascontiguousarray(x0[sl]), STAR_SETS[r], T, dtype=np.float64)
        rv = ref[tuple(i - s.start for i, s in zip(idx, sl))]
        errs.append(abs(float(got[idx]) - rv) / abs(rv))
    report(wl["name"], "forward, 2 cone samples", max(errs), "T=%d, radius %d" % (T, r), T)


def test_fp64_diffusion3d_512():
    wl = WORKLOADS["diffusion3d_512"]
    x0 = wl.field()
    got = gpu_run(wl, x0, None)
    idx = [(0, 0, 0), (511, 300, 7), (256, 255, 250)]
    errs = []
    for i in idx:
        r = cone64(x0, None, wl.coeffs, wl.T, i)
        errs.append(abs(float(got[i]) - r) / abs(r))
    report(wl.name, "forward, %d cone samples" % len(idx), max(errs), "T=%d" % wl.T, wl.T)


def test_fp64_hotspot3d_256_forward_and_adjoint():
    wl = WORKLOADS["hotspot3d_256_adjoint"]
    cf = wl.coeffs
    x0, p, y = wl.field(), wl.power(), wl.target()
    plan = S.Plan(HOTSPOT, wl.shape)
    try:
        x = torch.from_numpy(x0).cuda()
        pw = torch.from_numpy(p).cuda()
        plan.run_ckpt(x, cf, wl.T, wl.ckpt_every, pw)
        xT = x.cpu().numpy()
        g = (x - torch.from_numpy(y).cuda()).contiguous()
        gx = torch.empty_like(g)
        gp = torch.empty_like(g)
        plan.adjoint(g, cf, wl.T, gx, gp, pw, 0)
        torch.cuda.synchronize()
        gh, gxh, gph = g.cpu().numpy(), gx.cpu().numpy(), gp.cpu().numpy()
    finally:
        plan.close()
    ref = oracle.forward(x0, cf, wl.T, power=p, dtype=np.float64)
    report(wl.name, "forward x_T, all cells", maxrel(xT, ref), "T=%d" % wl.T, wl.T)
    # symmetric operator: grad_x0 = A^T g = linear part of the forward map applied to g
    lin = cf.copy()
    lin[7:] = 0.0
    ref_x = oracle.forward(gh.astype(np.float64), lin, wl.T, form=DIFFUSION, dtype=np.float64)
    err_x = float(np.max(np.abs(gxh - ref_x)) / np.max(np.abs(ref_x)))
    report(wl.name, "adjoint grad_x0 (normwise)", err_x, "T=%d, same cotangent" % wl.T, wl.T)
    src = cf.copy()
    src[8] = 0.0
    ref_p = oracle.forward(np.zeros_like(gh, dtype=np.float64), src, wl.T, power=gh.astype(np.float64),
                           form=HOTSPOT, dtype=np.float64)
    err_p = float(np.max(np.abs(gph - ref_p)) / np.max(np.abs(ref_p)))
    report(wl.name, "adjoint grad_p (normwise)", err_p, "T=%d, same cotangent" % wl.T, wl.T)


def test_fp64_batched_smallest_grids():
    grids = batch_grids()
    xs = [torch.from_numpy(g.field()).cuda() for g in grids]
    x0s = [x.cpu().numpy() for x in xs]
    cfs = [SETS[g.coef_set] for g in grids]
    S.run_batched(xs, cfs, [g.T for g in grids])
    torch.cuda.synchronize()
    # the smallest 2D and the smallest 3D grid of the batch, whole grids
    picks = [min((i for i, g in enumerate(grids) if g.ndim == d), key=lambda i: grids[i].nx) for d in (2, 3)]
    for i in picks:
        g = grids[i]
        ref = oracle.forward(x0s[i], cfs[i], g.T, dtype=np.float64)
        report("batched_64[%d]" % i, "%dD side %d, all cells" % (g.ndim, g.nx), maxrel(xs[i].cpu().numpy(), ref),
               "T=%d" % g.T, g.T)
