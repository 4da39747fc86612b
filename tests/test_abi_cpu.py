"""CPU-side checks of the C ABI: the library loads, exports every declared entry point,
validates arguments before touching a device, and its performance model (paper Section 4,
Eq. 3-9) reproduces the paper's own estimates (Table 4 "Estimated Performance", Table 6)."""
import csv
import ctypes
import os
import re

import pytest

import paper_1802_00438_amd as S

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
GOLDEN = os.path.join(ROOT, "tests", "golden")


@pytest.fixture(scope="module", autouse=True)
def built_library():
    if not os.path.exists(S.library_path()):
        from paper_1802_00438_amd import build as B
        B.build(force=False)
    yield


def test_library_exports_every_declared_symbol():
    header = open(os.path.join(ROOT, "include", "stencil.h")).read()
    declared = set(re.findall(r"\b(stencil_[a-z_]+)\s*\(", header))
    assert declared == set(S.EXPORTED)
    L = S.lib()
    for name in declared:
        assert getattr(L, name) is not None


def test_status_strings():
    for code, name in S.STATUS.items():
        assert S.stencil_status_string(code) == name
    assert S.stencil_status_string(42) == "STENCIL_ERR_UNKNOWN"


@pytest.mark.parametrize("args", [
    (S.DIFFUSION, 4, 8, 8, 1),   # bad ndim
    (S.DIFFUSION, 2, 0, 8, 1),   # empty
    (S.DIFFUSION, 2, 8, -1, 1),
    (S.DIFFUSION, 2, 8, 8, 2),   # 2D with nz != 1
    (S.DIFFUSION, 3, 8, 8, 0),
    (7, 2, 8, 8, 1),             # unknown form
])
def test_create_rejects_bad_shapes(args):
    L = S.lib()
    h = ctypes.c_void_p(1234)
    st = L.stencil_create(ctypes.byref(h), *args, None, None)
    assert st == -1
    assert h.value is None
    assert S.stencil_last_error()


def test_create_rejects_bad_tuning():
    L = S.lib()
    h = ctypes.c_void_p()
    t = S.Tuning(variant=5)
    assert L.stencil_create(ctypes.byref(h), 0, 2, 8, 8, 1, ctypes.byref(t), None) == -1
    t = S.Tuning(k=-1)
    assert L.stencil_create(ctypes.byref(h), 0, 2, 8, 8, 1, ctypes.byref(t), None) == -1
    t = S.Tuning(vec=3)
    assert L.stencil_create(ctypes.byref(h), 0, 2, 8, 8, 1, ctypes.byref(t), None) == -2
    assert L.stencil_create(None, 0, 2, 8, 8, 1, None, None) == -1


def test_calls_on_null_plan_are_rejected():
    L = S.lib()
    c = S.make_coeffs([0.5, 0.125, 0.125, 0.125, 0.125])
    assert L.stencil_run(None, None, None, ctypes.byref(c), 1) == -1
    assert L.stencil_run_ckpt(None, None, None, ctypes.byref(c), 1, 0) == -1
    assert L.stencil_adjoint(None, None, None, ctypes.byref(c), 1, None, None, 0) == -1
    assert L.stencil_get_tuning(None, None) == -1
    m = S.PlanModel()
    assert L.stencil_plan_model(None, 10, ctypes.byref(m)) == -1
    w = (ctypes.c_float * 9)(*([0.5] + [0.0625] * 8))
    assert L.stencil_run_star(None, None, w, 1) == -1
    L.stencil_destroy(None)        # no-op
    L.stencil_batch_destroy(None)  # no-op


def test_batched_validates_items_before_device_work():
    L = S.lib()
    c = S.make_coeffs([0.5, 0.125, 0.125, 0.125, 0.125])
    bad = [
        S.BatchItem(S.HOTSPOT, 2, 8, 8, 1, 4096, None, c, 3),  # hotspot: unsupported
        S.BatchItem(S.DIFFUSION, 2, 8, 8, 1, None, None, c, 3),  # null grid
        S.BatchItem(S.DIFFUSION, 2, 8, 8, 1, 4098, None, c, 3),  # misaligned
        S.BatchItem(S.DIFFUSION, 2, 8, 8, 1, 4096, None, c, -1),  # T < 0
        S.BatchItem(S.DIFFUSION, 3, 8, 0, 8, 4096, None, c, 3),  # empty
    ]
    for item, code in zip(bad, (-2, -1, -1, -1, -1)):
        arr = (S.BatchItem * 1)(item)
        assert L.stencil_run_batched(1, arr, None, None) == code
    dup = (S.BatchItem * 2)(S.BatchItem(0, 2, 8, 8, 1, 4096, None, c, 1), S.BatchItem(0, 2, 8, 8, 1, 4096, None, c, 1))
    assert L.stencil_run_batched(2, dup, None, None) == -1
    nan = S.make_coeffs([float("nan"), 0, 0, 0, 0])
    arr = (S.BatchItem * 1)(S.BatchItem(0, 2, 8, 8, 1, 4096, None, nan, 1))
    assert L.stencil_run_batched(1, arr, None, None) == -1
    assert L.stencil_run_batched(-1, None, None, None) == -1


def _rows(name):
    with open(os.path.join(GOLDEN, name)) as f:
        return list(csv.DictReader(l for l in f if not l.startswith("#")))


TABLE2 = {r["stencil"]: r for r in _rows("paper_table2.csv")}


def _estimate(stencil, bsize, par_vec, par_time, dim, fmax_hz, th_max, iters):
    t2 = TABLE2[stencil]
    nd = int(t2["ndim"])
    return S.stencil_model_estimate(
        ndim=nd, rad=1, par_vec=par_vec, par_time=par_time, f_max_hz=fmax_hz, size_cell=4,
        num_read=int(t2["num_read"]), num_write=int(t2["num_write"]), bsize_x=bsize,
        bsize_y=bsize if nd == 3 else 0, dim_x=dim, dim_y=dim, dim_z=dim if nd == 3 else 1, iter=iters,
        th_max_gbs=th_max)


@pytest.mark.parametrize("row", _rows("paper_table4.csv"), ids=lambda r: "%s-%s-%s" % (r["stencil"], r["device"], r["par_time"]))
def test_model_reproduces_table4_estimates(row):
    th = 25.6 if row["device"] == "S-V" else 34.128  # Table 3 peaks (A-10: 2 x DDR4-2133 x 8 B)
    r = _estimate(row["stencil"], int(row["bsize"]), int(row["par_vec"]), int(row["par_time"]), int(row["dim"]),
                  float(row["fmax_mhz"]) * 1e6, th, 1000)
    est = float(row["estimated_gbs"])
    assert abs(r["throughput_gbs"] - est) / est < 1e-5


@pytest.mark.parametrize("row", _rows("paper_table4.csv"), ids=lambda r: "%s-%s-%s" % (r["stencil"], r["device"], r["par_time"]))
def test_table4_unit_conversions(row):
    """GFLOP/s = GB/s x FLOP/Byte and GCell/s = GB/s / Bytes-per-update (Table 2)."""
    t2 = TABLE2[row["stencil"]]
    gbs = float(row["measured_gbs"])
    assert abs(gbs / float(t2["bytes_pcu"]) - float(row["measured_gcells"])) < 1.5e-3
    assert abs(gbs * float(t2["flop_pcu"]) / float(t2["bytes_pcu"]) - float(row["measured_gflops"])) < 1.5e-3


@pytest.mark.parametrize("row", _rows("paper_table6.csv"), ids=lambda r: "%s-%s" % (r["fpga"], r["stencil"]))
def test_model_reproduces_table6_projections(row):
    r = _estimate(row["stencil"], int(row["bsize"]), int(row["par_vec"]), int(row["par_time"]), int(row["dim"]),
                  float(row["fmax_mhz"]) * 1e6, float(row["th_max_gbs"]), 5000)
    t2 = TABLE2[row["stencil"]]
    gbs = r["throughput_gbs"] * float(row["calibration"])
    assert abs(gbs - float(row["gbs"])) < 0.051
    gflops = gbs * float(t2["flop_pcu"]) / float(t2["bytes_pcu"])
    assert abs(gflops - float(row["gflops"])) < 0.051
    assert abs(r["th_mem_gbs"] - float(row["used_bw_gbs"])) < 0.051


def test_model_rejects_bad_parameters():
    with pytest.raises(S.StencilError):
        S.stencil_model_estimate(ndim=2, rad=1, par_vec=4, par_time=3000, f_max_hz=3e8, size_cell=4, num_read=1,
                                 num_write=1, bsize_x=4096, bsize_y=0, dim_x=100, dim_y=100, dim_z=1, iter=10,
                                 th_max_gbs=10.0)
    with pytest.raises(S.StencilError):
        S.stencil_model_estimate(ndim=5, rad=1, par_vec=4, par_time=3, f_max_hz=3e8, size_cell=4, num_read=1,
                                 num_write=1, bsize_x=4096, bsize_y=0, dim_x=100, dim_y=100, dim_z=1, iter=10,
                                 th_max_gbs=10.0)


def test_binding_fails_loudly_without_library(tmp_path, monkeypatch):
    import importlib
    mod = importlib.import_module("paper_1802_00438_amd")
    monkeypatch.setattr(mod, "LIB_PATH", str(tmp_path / "missing.so"))
    monkeypatch.setattr(mod, "_lib", None)
    with pytest.raises(ImportError):
        mod.lib()


def test_create_star_rejects_bad_arguments_before_device_work():
    L = S.lib()
    h = ctypes.c_void_p(1234)
    assert L.stencil_create_star(ctypes.byref(h), 4, 2, 8, 8, 8, None, None) == -1  # ndim 2 or 3
    assert h.value is None
    assert L.stencil_create_star(ctypes.byref(h), 3, 5, 8, 8, 8, None, None) == -2  # 3D rad > 4
    assert L.stencil_create_star(ctypes.byref(h), 2, 0, 8, 8, 1, None, None) == -1  # rad < 1
    assert L.stencil_create_star(ctypes.byref(h), 2, 5, 8, 8, 1, None, None) == -2  # rad > 4
    t = S.Tuning(variant=3)
    assert L.stencil_create_star(ctypes.byref(h), 2, 2, 8, 8, 1, ctypes.byref(t), None) == -1
    assert L.stencil_create_star(None, 2, 2, 8, 8, 1, None, None) == -1


def test_noalloc_batch_rejects_bad_arguments_before_device_work():
    """Argument errors of the no-allocation batched launch return before any device call."""
    L = S.lib()
    item = S.BatchItem(S.DIFFUSION, 2, 8, 8, 1, 4096, None, S.make_coeffs([0.5, 0.125, 0.125, 0.125, 0.125]), 3)
    arr = (S.BatchItem * 1)(item)
    assert L.stencil_run_batched_noalloc(1, arr, None, None) == -1          # no partner list
    parr = (ctypes.c_void_p * 1)(None)
    assert L.stencil_run_batched_noalloc(1, arr, parr, None) == -1          # NULL partner
    parr = (ctypes.c_void_p * 1)(4096)
    assert L.stencil_run_batched_noalloc(1, arr, parr, None) == -1          # partner aliases the grid
    parr = (ctypes.c_void_p * 1)(8194)
    assert L.stencil_run_batched_noalloc(1, arr, parr, None) == -1          # misaligned partner
    bad = (S.BatchItem * 1)(S.BatchItem(S.HOTSPOT, 2, 8, 8, 1, 4096, None, S.make_coeffs([0.5]), 3))
    assert L.stencil_run_batched_noalloc(1, bad, (ctypes.c_void_p * 1)(65536), None) == -2  # hotspot
    assert L.stencil_run_batched_noalloc(-1, None, None, None) == -1


def test_star_hotspot_rejects_bad_arguments_before_device_work():
    L = S.lib()
    w = (ctypes.c_float * 9)(*([0.2] * 9))
    src = (ctypes.c_float * 3)(0.125, 0.25, 64.0)
    assert L.stencil_run_star_hotspot(None, None, None, w, src, 1) == -1  # no plan
    assert L.stencil_run_star_hotspot(None, None, None, None, None, 1) == -1


def test_star_adjoint_rejects_bad_arguments_before_device_work():
    L = S.lib()
    w = (ctypes.c_float * 9)(*([0.2] * 9))
    assert L.stencil_adjoint_star(None, None, w, None, 1, None, None) == -1  # no plan
