"""Host logic that runs without a GPU: the bench's tile geometry and algorithmic byte counts,
and the binding's argument checks (which raise before any library call)."""
import math

import numpy as np
import pytest

import bench
import paper_1802_00438_amd as S
from workloads import SETS, STAR_SETS, batch_grids, star_weights


def test_tb2d_geometry_covers_the_grid():
    for nx, ny, K, seg in [(16384, 16384, 12, 192), (1001, 97, 8, 30), (256, 256, 4, 8), (7, 5, 16, 100)]:
        W, kr, cs, ntx, sg, nseg = bench.tb2d_geometry(nx, ny, K, seg)
        assert W == 256 and kr % 4 == 0 and kr >= K and cs % 4 == 0 and cs > 0
        assert W - kr - cs >= K  # right halo
        assert (ntx - 1) * cs < nx <= ntx * cs
        assert (nseg - 1) * sg < ny <= nseg * sg


def test_interior_rectangle_is_edge_free():
    nx = ny = 16384
    K, seg = 12, 192
    W, kr, cs, ntx, sg, nseg = bench.tb2d_geometry(nx, ny, K, seg)
    xs, ys = bench.tb2d_interior(nx, ny, K, K, seg)
    assert (len(xs), len(ys)) == (69, 84)
    for tx in range(ntx):
        ws = tx * cs - kr
        assert (tx in xs) == (ws >= 0 and ws + W <= nx)
    for s in range(nseg):
        r0, r1 = s * sg, min(s * sg + sg, ny)
        assert (s in ys) == (r0 - K > 0 and r1 + K < ny)


def test_run_roofline_of_radius_one_matches_the_pass_count():
    """run_roofline sums one pass per k steps plus a shorter last one; for radius 1 its bytes
    equal tb2d_bytes_flops over all tiles, pass by pass."""
    ms = 100.0
    r = bench.run_roofline(16384, 16384, 1000, 12, bench.smallest_at_least([4, 8, 12, 16]), 192, 1, 2, 10, ms)
    b12, f12 = bench.tb2d_bytes_flops(16384, 16384, 12, 12, 192, hot=True)
    b4, f4 = bench.tb2d_bytes_flops(16384, 16384, 4, 4, 192, hot=True)
    total_b = 83 * b12 + b4
    assert abs(r["frac_hbm"] - total_b / (ms * 1e-3) / 1e9 / bench.HBM_PEAK_GBS) < 1e-4
    assert r["bound"] in ("alu", "hbm")
    assert bench.smallest_at_least([1, 2, 4, 8])(3) == 4 and bench.smallest_at_least([1, 2, 4])(7) == 4


def test_star_weight_layout_and_sets():
    w = star_weights(0.5, [0.1, 0.2], [0.3, 0.4], [0.01, 0.02], [0.03, 0.04])
    assert list(np.round(w, 6)) == [0.5, 0.1, 0.3, 0.2, 0.4, 0.01, 0.02, 0.03, 0.04]
    for r, ws in STAR_SETS.items():
        assert ws.size == 1 + 4 * r and float(ws.astype(np.float64).sum()) == 1.0


def test_batch_recipe_is_deterministic():
    a = batch_grids()
    b = batch_grids()
    assert [(g.nx, g.T) for g in a] == [(g.nx, g.T) for g in b]
    assert sum(g.ndim == 2 for g in a) == 48 and sum(g.ndim == 3 for g in a) == 16
    assert all(256 <= g.nx <= 4096 for g in a if g.ndim == 2)
    assert all(64 <= g.nx <= 256 for g in a if g.ndim == 3)
    assert all(50 <= g.T <= 500 for g in a)


def test_binding_rejects_host_tensors_before_any_library_call():
    torch = pytest.importorskip("torch")
    x = torch.zeros(8, 8)  # a CPU tensor
    with pytest.raises(ValueError):
        S.run(x, SETS["D2"], 1)
    with pytest.raises(ValueError):
        S._check_tensor(torch.zeros(8, 8, dtype=torch.float64), "x")
