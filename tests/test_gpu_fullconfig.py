"""Parity at the full configurations the bench times, element by element.

* The 64-grid batch: every grid of the real batch (its true sizes, step counts and the
  launch configuration the bench replays) against the FP32 oracle, on the first launch and
  on a graph replay.
* Hotspot 2D 16384^2, T = 1000, on the auto-tuned blocking the bench runs: whole-width bands
  of output rows at the top edge, across a tile-segment seam in mid-grid and at the bottom
  edge, so that every x-tile seam, the edge-tile frame and the interior tiles of the split pass
  are compared cell by cell.
* Diffusion 3D 512^3, T = 200, auto-tuned: whole 512^2 planes in mid-grid and at both z edges.

A cell after T steps depends only on the initial cells within T steps of it (radius 1), so
the oracle reproduces a band of rows (planes) exactly from the band widened by T on each side
and cut at the real grid edges: an artificial cut needs T steps to reach the band.  The FP32
oracle then performs the very operations the full-grid run performs on those cells, so the
GPU result is expected bit for bit; max-rel <= 1e-5 is asserted as well.
"""
import numpy as np
import pytest

import oracle
import paper_1802_00438_amd as S
from workloads import WORKLOADS, SETS, DIFFUSION, HOTSPOT, batch_grids

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL = 1e-5


def maxrel(got, ref):
    ref = np.asarray(ref, dtype=np.float64)
    return float(np.max(np.abs(np.asarray(got, dtype=np.float64) - ref) / np.maximum(np.abs(ref), 1e-30)))


def assert_equal_cells(got, ref, what):
    assert got.shape == ref.shape, what
    err = maxrel(got, ref)
    assert err <= TOL, (what, err)
    bad = np.flatnonzero(got.ravel() != ref.ravel())
    assert bad.size == 0, (what, bad.size, np.unravel_index(bad[0], got.shape) if bad.size else None)


def band_reference(x0, power, cf, T, lo, hi, axis0_len):
    """Oracle rows (2D) / planes (3D) [lo, hi) after T steps, from the band widened by T."""
    a, b = max(0, lo - T), min(axis0_len, hi + T)
    sub = np.ascontiguousarray(x0[a:b])
    psub = None if power is None else np.ascontiguousarray(power[a:b])
    out = oracle.forward(sub, cf, T, power=psub, dtype=np.float32)
    return out[lo - a:hi - a]


def test_batched_64_every_grid_first_launch_and_replay():
    grids = batch_grids()
    x0s = [g.field() for g in grids]
    xs = [torch.from_numpy(x).cuda() for x in x0s]
    cfs = [SETS[g.coef_set] for g in grids]
    ts = [g.T for g in grids]
    cache = S.run_batched(xs, cfs, ts)  # builds, captures and runs the graph once
    try:
        torch.cuda.synchronize()
        first = [x.cpu().numpy() for x in xs]
        # replay on the same buffers, reloaded with the initial fields
        for x, h in zip(xs, x0s):
            x.copy_(torch.from_numpy(h))
        S.run_batched(xs, cfs, ts, cache=cache)
        torch.cuda.synchronize()
        replay = [x.cpu().numpy() for x in xs]
    finally:
        S.stencil_batch_destroy(cache)
    for i, g in enumerate(grids):
        ref = oracle.forward(x0s[i], cfs[i], g.T, dtype=np.float32)
        what = "grid %d: %dD side %d, T=%d" % (i, g.ndim, g.nx, g.T)
        assert_equal_cells(first[i], ref, what + " (first launch)")
        assert_equal_cells(replay[i], ref, what + " (replay)")


def test_hotspot2d_16384_full_width_bands_across_seams():
    wl = WORKLOADS["hotspot2d_16384"]
    x0 = wl.field()
    p = wl.power()
    x = torch.from_numpy(x0).cuda()
    pw = torch.from_numpy(p).cuda()
    plan = S.Plan(HOTSPOT, wl.shape)  # auto-tuned, as the bench runs it
    try:
        seg = plan.tuning["seg_len"]
        plan.run(x, wl.coeffs, wl.T, pw)
        torch.cuda.synchronize()
        got = x.cpu().numpy()
    finally:
        plan.close()
    ny = wl.ny
    seam = (ny // 2) // seg * seg  # a segment boundary in mid-grid
    bands = [(0, min(ny, 2 * seg + 64)), (seam - 32, seam + 32), (ny - 64, ny)]
    for lo, hi in bands:
        ref = band_reference(x0, p, wl.coeffs, wl.T, lo, hi, ny)
        assert_equal_cells(got[lo:hi], ref, "rows [%d, %d), seg %d" % (lo, hi, seg))


def test_diffusion3d_512_whole_planes():
    wl = WORKLOADS["diffusion3d_512"]
    x0 = wl.field()
    x = torch.from_numpy(x0).cuda()
    plan = S.Plan(DIFFUSION, wl.shape)  # auto-tuned, as the bench runs it
    try:
        plan.run(x, wl.coeffs, wl.T)
        torch.cuda.synchronize()
        got = x.cpu().numpy()
    finally:
        plan.close()
    nz = wl.nz
    for lo, hi in [(0, 6), (250, 262), (nz - 6, nz)]:
        ref = band_reference(x0, None, wl.coeffs, wl.T, lo, hi, nz)
        assert_equal_cells(got[lo:hi], ref, "planes [%d, %d)" % (lo, hi))
