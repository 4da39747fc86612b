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


def test_tb2d_pass_counts_window_rows_and_outputs():
    """Bytes of one pass: every tile reads its 256-column window over seg + 2k rows per field and
    writes its output cells once; the interior part is a subset of the whole pass."""
    b, f = bench.tb2d_pass(16384, 16384, 12, 12, 192, 2, 10)
    W, kr, cs, ntx, sg, nseg = bench.tb2d_geometry(16384, 16384, 12, 192)
    assert b == ntx * nseg * (192 + 24) * 256 * 4 * 2 + 16384 * 16384 * 4
    assert f == ntx * nseg * 256 * (192 + 12) * 12 * 10
    bi, fi = bench.tb2d_pass(16384, 16384, 12, 12, 192, 2, 10, interior_only=True)
    assert bi < b and fi < f and bi == 69 * 84 * 216 * 256 * 8 + 69 * cs * 84 * 192 * 4
    assert bench.tb2d_split(16384, 16384, 12, 12, 192) and not bench.tb2d_split(256, 256, 4, 4, 256)


def test_tb3d_geometry_and_segments():
    # 512^3 at k = 4 in 128 x 48 windows: 5 x 13 edge-flush tiles; 256^3 at k = 3: 3 x 6
    assert bench.tb3d_geometry(4, 512, 512) == (5, 13)
    assert bench.tb3d_geometry(3, 256, 256) == (3, 6)
    assert bench.tb3d_geometry(2, 100, 40) == (1, 1)  # narrower than a window: uniform tiling
    for nwork, segz in ((256, 0), (0, 64), (0, 1000)):
        segs = bench.tb3d_segments(65, 512, nwork, segz)
        assert sum(ze - zs for zs, ze in segs) == 65 * 512  # every (column, plane) unit once
        assert all(0 <= zs < ze <= 512 for zs, ze in segs)
    segs = bench.tb3d_segments(10, 72, 7, 0, zlo=4, zhi=68)
    assert sum(ze - zs for zs, ze in segs) == 10 * 64 and all(4 <= zs < ze <= 68 for zs, ze in segs)
    tun = {"bsize_x": 128, "bsize_y": 48, "nwork": 256, "seg_len": 130}
    b, f = bench.tb3d_pass(512, 512, 512, 4, 4, tun, 1, 4, 13)
    assert 512 ** 3 * 4 * 1.5 < b < 512 ** 3 * 4 * 3.2  # reads 1.5-2x the grid, writes it once
    assert f > 512 ** 3 * 4 * 13


def test_roofline_record_picks_the_larger_fraction():
    r = bench.roofline("k", "plain", {}, 1.0, 4.0e9, 1.0e9, 5000.0)
    assert r["bound"] == "hbm" and abs(r["frac"] - 0.5) < 1e-9 and abs(r["frac_copy_bw"] - 0.8) < 1e-9
    assert r["traffic"] is None
    r = bench.roofline("k", "plain", {}, 1.0, 1.0e9, 70.0e9, 5000.0)
    assert r["bound"] == "alu" and abs(r["achieved"] - 70.0) < 1e-6
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


def test_star3d_pass_counts_windows_and_pipeline():
    """A grid inside one window and one segment is read once and written once; the 512^3
    radius-2 pass reads each cell about (64/56)^2 x (103+8)/103 times."""
    b, f = bench.star3d_pass(9, 7, 5, 1, 1, 100)
    assert b == 9 * 7 * 5 * 4 * 2
    assert f == ((5 + 3 + 2) // 3 * 3) * 64 * 64 * 13
    b, f = bench.star3d_pass(512, 512, 512, 2, 2, 103)
    cs = 64 - 8
    ntx = math.ceil(512 / cs)
    reads = b / (512 ** 3 * 4) - 1.0
    assert (64 / cs) ** 2 < reads < (64 / cs) ** 2 * (103 + 8) / 103 * 1.01
    assert f == sum(((min(z + 103, 512) - z) + 10 + 2) // 3 * 3 for z in range(0, 512, 103)) * ntx * ntx * 4096 * 2 * 25


def test_counter_records_parse_the_committed_summaries():
    """Every counter summary under profiles/ yields its records (the list sits in a fenced
    json block), each with the fields measured_traffic needs."""
    recs = bench.counter_records()
    assert recs, "no counter records found under profiles/"
    for r in recs:
        for key in ("kernel", "family", "config", "source_hash", "fetch_kib_per_dispatch",
                    "write_kib_per_dispatch", "copy_fetch_factor", "copy_write_factor"):
            assert key in r, (r.get("kernel"), key)
        assert r["family"] in bench.KERNEL_SOURCES


def test_measured_traffic_needs_current_sources_and_the_same_config(monkeypatch):
    fam = "plain"
    rec = {"kernel": "plain_kernel<true, false, false, false>", "family": fam, "config": {"shape": [64, 64]},
           "source_hash": bench.source_hash(bench.KERNEL_SOURCES[fam]), "fetch_kib_per_dispatch": 2.0,
           "write_kib_per_dispatch": 3.0, "copy_fetch_factor": 0.5, "copy_write_factor": 1.0}
    monkeypatch.setattr(bench, "counter_records", lambda: [rec])
    sym = rec["kernel"]
    assert bench.measured_traffic(sym, fam, {"shape": [64, 64]}) == 2.0 * 1024 / 0.5 + 3.0 * 1024
    assert bench.measured_traffic(sym, fam, {"shape": [64, 128]}) is None
    assert bench.measured_traffic("plain_kernel<false, false, false, false>", fam, {"shape": [64, 64]}) is None
    monkeypatch.setattr(bench, "counter_records", lambda: [dict(rec, source_hash="0" * 16)])
    assert bench.measured_traffic(sym, fam, {"shape": [64, 64]}) is None
