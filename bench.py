"""Benchmark: temporal-blocked hotspot 2D, 16384 x 16384 cells, 1000 time steps, one MI355X.

One "step" of this bench is one whole run of the hot path: stencil_run over the 16384^2
hotspot grid for T = 1000 time steps (all passes, boundary handling, ping-pong), with the
temperature and power maps already resident in HBM.  value = cell updates per second
(GCell/s); the single-pass HBM roofline of this stencil is 8 TB/s / 12 B = 667 GCell/s
(Table 2 bytes per update).

The same JSON line carries, for the dominant kernel and for the dominant kernel of every other
workload (unless --quick), a roofline record: algorithmic HBM bytes and executed FP32 FLOPs
per launch over the kernel's average launch duration, measured here with HIP events on the
stream the kernel runs on, against the HBM peak (8 TB/s), the plain-FP32 ALU peak (78.6
TFLOP/s) and the device-to-device copy bandwidth measured in the same run.  `traffic` is the
HBM traffic the committed counter summaries in profiles/ record for the same kernel build and
configuration (null otherwise).  The CPU oracle is timed on a bounded sample.  `model_accuracy`
sets each workload against the library's own time model and the paper's Eq. 3-9 model.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--quick] [--only a,b] [--no-cpu]
"""
import argparse
import glob
import hashlib
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)
CSRC = os.path.join(ROOT, "paper_1802_00438_amd", "csrc")

HBM_PEAK_GBS = 8000.0
# 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz x 2 FLOP per FMA, plain (non-packed) FP32: the kernels
# are built without packed FP32, so the 157.3 TFLOP/s packed figure is out of their reach
ALU_PEAK_TFLOPS = 256 * 4 * 16 * 2.4e9 * 2 / 1e12

SECONDARY = ["plain_hotspot2d_16384", "hotspot2d_phys_16384", "star2d_r2_16384", "star3d_r2_512", "diffusion3d_512",
             "diffusion2d_256", "hotspot3d_256", "batched_64", "slab3d_512x512x64"]


def log(msg):
    print(msg, file=sys.stderr, flush=True)


# ------------------------------------------------------------------ launch geometry
# These mirror the host planner of the library (the same formulas), so that bytes and FLOPs per
# launch can be counted from the blocking a plan reports.

def tb2d_geometry(nx, ny, K, seg, R=1):
    """2D pass: 256-column windows with a left halo kr (R*K rounded up to 4) and cs output
    columns, by `seg`-row segments."""
    W = 256
    kr = (R * K + 3) // 4 * 4
    cs = (W - R * K - kr) // 4 * 4
    seg = max(1, min(seg, ny))
    return W, kr, cs, math.ceil(nx / cs), seg, math.ceil(ny / seg)


def tb2d_interior(nx, ny, K, keff, seg):
    """Interior rectangle of tiles (window inside the grid in x, rows clear of the first and
    last grid row): the tiles the edge-free kernel runs when a pass is split."""
    W, kr, cs, ntx, seg, nseg = tb2d_geometry(nx, ny, K, seg)
    xs = [tx for tx in range(ntx) if tx * cs - kr >= 0 and tx * cs - kr + W <= nx]
    ys = [sg for sg in range(nseg) if sg * seg - keff > 0 and min(sg * seg + seg, ny) + keff < ny]
    if not xs or not ys:
        return [], []
    return list(range(xs[0], xs[-1] + 1)), list(range(ys[0], ys[-1] + 1))


def tb2d_split(nx, ny, K, keff, seg):
    """Whether a pass splits into the edge-free kernel and the frame kernel."""
    xs, ys = tb2d_interior(nx, ny, K, keff, seg)
    n = len(xs) * len(ys)
    _, _, _, ntx, _, nseg = tb2d_geometry(nx, ny, K, seg)
    return n >= 1024 and n < ntx * nseg and nx % 4 == 0


def tb2d_pass(nx, ny, K, keff, seg, nread, flops_per, interior_only=False, R=1):
    """Algorithmic HBM bytes and executed FLOPs of one temporal-blocked 2D pass with keff fused
    steps (or of its interior tiles only): every window row of a tile is read once per pass
    (temperature, plus power for hotspot), every output cell is written once; every lane of the
    window computes every level of the rows it streams (seg + R*keff rows, halos included)."""
    W, kr, cs, ntx, seg, nseg = tb2d_geometry(nx, ny, K, seg, R)
    if interior_only:
        xs, ys = tb2d_interior(nx, ny, K, keff, seg)
    else:
        xs, ys = list(range(ntx)), list(range(nseg))
    tiles = len(xs) * len(ys)
    out_cells = sum(min(cs, nx - tx * cs) for tx in xs) * sum(min(seg, ny - sg * seg) for sg in ys)
    bytes_ = tiles * (seg + 2 * R * keff) * W * 4 * nread + out_cells * 4
    flops = tiles * W * (seg + R * keff) * keff * flops_per
    return bytes_, flops


def tb3d_geometry(K, nx, ny, WX=128, WY=48):
    """Tiles along x and y of a 3D pass (edge-flush tiling where the grid is at least one window
    wide or high; one window flush with x = 0 where an even grid is narrower than a window;
    else uniform tiling)."""
    krx = (K + 1) // 2 * 2
    csx = (WX - K - krx) // 2 * 2
    csy = WY - 2 * K
    if nx >= WX and nx % 2 == 0:
        fx = (WX - K) // 2 * 2
        ntx = 1 if nx == WX else (2 if nx <= 2 * fx else 2 + math.ceil((nx - 2 * fx) / csx))
    elif nx % 2 == 0:
        ntx = 1
    else:
        ntx = math.ceil(nx / csx)
    if ny >= WY:
        fy = WY - K
        nty = 1 if ny == WY else (2 if ny <= 2 * fy else 2 + math.ceil((ny - 2 * fy) / csy))
    else:
        nty = math.ceil(ny / csy)
    return ntx, nty


def tb3d_segments(ncols, nz, nwork, segz, zlo=0, zhi=None):
    """Column segments (zs, ze) of one 3D pass: nwork > 0, the balanced launch (each workgroup
    streams an equal share of all (column, plane) units); else one tile per segz planes."""
    zhi = nz if zhi is None else zhi
    nzo = zhi - zlo
    out = []
    if nwork > 0:
        units = ncols * nzo
        for w in range(nwork):
            u, u1 = units * w // nwork, units * (w + 1) // nwork
            while u < u1:
                col = u // nzo
                zs = u - col * nzo
                ze = min(nzo, zs + (u1 - u))
                out.append((zlo + zs, zlo + ze))
                u += ze - zs
    else:
        segz = max(1, min(segz, nzo))
        for _ in range(ncols):
            for zs in range(zlo, zhi, segz):
                out.append((zs, min(zs + segz, zhi)))
    return out


def tb3d_pass(nx, ny, nz, K, keff, tun, nread, out_bytes_per_cell, flops_per, zlo=0, zhi=None):
    """Algorithmic HBM bytes and executed FLOPs of one temporal-blocked 3D pass: each column
    segment reads its window (WX x WY) of the planes within keff of its output planes, inside
    the grid, once (nread fields); every output cell is written (out_bytes_per_cell); every
    lane computes every level of every plane it streams (the pipeline runs output planes +
    keff + K iterations, rounded up to even)."""
    WX, WY = tun["bsize_x"], tun["bsize_y"]
    ntx, nty = tb3d_geometry(K, nx, ny, WX, WY)
    segs = tb3d_segments(ntx * nty, nz, tun["nwork"], tun["seg_len"], zlo, zhi)
    planes_read = sum(min(ze + keff, nz) - max(zs - keff, 0) for zs, ze in segs)
    iters = sum(((ze - zs) + keff + K + 1) // 2 * 2 for zs, ze in segs)
    zhi = nz if zhi is None else zhi
    bytes_ = planes_read * WX * WY * 4 * nread + nx * ny * (zhi - zlo) * out_bytes_per_cell
    flops = iters * WX * WY * K * flops_per
    return bytes_, flops


def star3d_pass(nx, ny, nz, R, K, segz):
    """Algorithmic HBM bytes and executed FLOPs of one radius-R 3D star pass fusing K steps:
    every tile reads its 64 x 64 window (inside the grid) over the planes within R*K of its
    output planes (inside the grid) once, and writes its output cells once; every lane computes
    K levels of its window cells for each pipeline iteration (output planes + K(2R+1), rounded
    up to a multiple of 3), at 12R + 1 FLOP per cell and level (a multiply and 6R FMAs)."""
    W, H = 64, R * K
    cs = W - 2 * H
    ntx, nty = math.ceil(nx / cs), math.ceil(ny / cs)
    segz = max(1, min(segz, nz))
    nsegz = math.ceil(nz / segz)
    cols = 0
    for tx in range(ntx):
        xw = tx * cs - H
        wx = min(xw + W, nx) - max(xw, 0)
        for ty in range(nty):
            yw = ty * cs - H
            cols += wx * (min(yw + W, ny) - max(yw, 0))
    iters = 0
    for sz in range(nsegz):
        z0, z1 = sz * segz, min(sz * segz + segz, nz)
        iters += ((z1 - z0) + K * (2 * R + 1) + 2) // 3 * 3
    bytes_ = sum(cols * (min(min(sz * segz + segz, nz) + H, nz) - max(sz * segz - H, 0)) for sz in range(nsegz)) * 4
    bytes_ += nx * ny * nz * 4
    flops = iters * ntx * nty * W * W * K * (12 * R + 1)
    return bytes_, flops


# ------------------------------------------------------------------ measured traffic records

def source_hash(files):
    h = hashlib.sha256()
    for f in files:
        with open(os.path.join(CSRC, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


KERNEL_SOURCES = {
    "tb2d_hot": ["tb2d.hpp", "device_common.hpp", "k_tb2d_hot.hip"],
    "tb2d_diff": ["tb2d.hpp", "device_common.hpp", "k_tb2d_diff.hip"],
    "tb2d_phys": ["tb2d.hpp", "device_common.hpp", "k_tb2d_phys.hip"],
    "star2d": ["star2d.hpp", "device_common.hpp", "k_star2d.hip", "k_star2d_r12.hip"],
    "star3d": ["star3d.hpp", "star2d.hpp", "device_common.hpp", "k_star3d.hip"],
    "star_adj": ["star_adjoint.hpp", "star2d.hpp", "device_common.hpp", "k_star_adj.hip"],
    "tb3d_diff": ["tb3d.hpp", "device_common.hpp", "k_tb3d_diff.hip"],
    "tb3d_hot": ["tb3d.hpp", "device_common.hpp", "k_tb3d_hot.hip"],
    "tb3d_adj": ["tb3d.hpp", "device_common.hpp", "k_tb3d_adj.hip"],
    "plain": ["plain.hpp", "device_common.hpp", "kernels_plain.hip"],
    "batched": ["batched.hip", "tb2d.hpp", "tb3d.hpp", "device_common.hpp"],
}


def counter_records():
    """Every counter record of the committed summaries in profiles/ (a JSON list between
    counters-json markers): FETCH_SIZE and WRITE_SIZE per dispatch with their copy calibration,
    the kernel symbol, its configuration and the hash of its sources."""
    recs = []
    for path in sorted(glob.glob(os.path.join(ROOT, "profiles", "*.md"))):
        with open(path) as fh:
            text = fh.read()
        if "<!-- counters-json -->" not in text:
            continue
        blob = text.split("<!-- counters-json -->")[1].split("<!-- /counters-json -->")[0]
        # the list sits in a fenced block (```json ... ```): parse from its first bracket to its last
        starts = [i for i in (blob.find("["), blob.find("{")) if i >= 0]
        end = max(blob.rfind("]"), blob.rfind("}"))
        if not starts or end < 0:
            continue
        try:
            data = json.loads(blob[min(starts):end + 1])
        except ValueError:
            continue
        recs.extend(data if isinstance(data, list) else [data])
    return recs


def measured_traffic(symbol, family, config):
    """HBM bytes per launch of `symbol` from the committed counter records, or None when no
    record matches this kernel build (source hash) and configuration."""
    want = source_hash(KERNEL_SOURCES[family])
    for r in counter_records():
        if r.get("kernel") != symbol or r.get("source_hash") != want:
            continue
        if any(r.get("config", {}).get(k) != v for k, v in config.items()):
            continue
        return (r["fetch_kib_per_dispatch"] * 1024.0 / r["copy_fetch_factor"] +
                r["write_kib_per_dispatch"] * 1024.0 / r["copy_write_factor"])
    return None


def roofline(symbol, family, config, avg_ms, bytes_, flops, copy_gbs, note=None):
    """Roofline record of one kernel: algorithmic bytes and executed FLOPs per launch over its
    average launch duration, against the HBM and ALU peaks; `bound` is the larger fraction."""
    s = avg_ms * 1e-3
    gbs = bytes_ / s / 1e9
    tf = flops / s / 1e12
    fh, fa = gbs / HBM_PEAK_GBS, tf / ALU_PEAK_TFLOPS
    if fa >= fh:
        r = {"bound": "alu", "achieved": round(tf, 3), "peak": round(ALU_PEAK_TFLOPS, 1), "unit": "TFLOP/s",
             "frac": round(fa, 4)}
    else:
        r = {"bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(fh, 4)}
    tb = measured_traffic(symbol, family, config)
    r["traffic"] = None if tb is None else round(tb / s / 1e9, 1)
    r.update({"kernel": symbol, "config": config, "avg_launch_ms": round(avg_ms, 4),
              "algorithmic_bytes_per_launch": int(bytes_), "executed_flops_per_launch": int(flops),
              "traffic_bytes_per_launch": None if tb is None else int(tb),
              "hbm_gbs_algorithmic": round(gbs, 1), "tflops_executed": round(tf, 3),
              "frac_hbm": round(fh, 4), "frac_alu": round(fa, 4),
              "frac_copy_bw": round(gbs / copy_gbs, 4) if copy_gbs else None})
    if note:
        r["note"] = note
    return r


# ------------------------------------------------------------------ timing helpers

def time_call(fn, stream, reps):
    """Average time of fn (enqueued on `stream`) over reps calls, by HIP events on that stream."""
    import torch
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(reps):
        fn()
    e1.record(stream)
    e1.synchronize()
    return e0.elapsed_time(e1) / reps


def copy_bandwidth(x, stream):
    """Device-to-device copy of x (read + write bytes over time), after a warm-up copy."""
    import torch
    tmp = torch.empty_like(x)
    tmp.copy_(x)
    ms = time_call(lambda: tmp.copy_(x), stream, 5)
    del tmp
    return 2.0 * x.numel() * 4 / (ms * 1e-3) / 1e9, ms


def smallest_at_least(ks):
    return lambda k: min([K for K in ks if K >= k] or [max(ks)])


def model_row(S, plan, T, ms, ndim, nread, dims, bsize, rad=1):
    """Measured against modelled for one workload: the library's own plan model (the tuner's)
    and the paper's Eq. 3-9 external-memory model at this blocking, with the HBM peak as
    th_max and one cell per lane per clock as the pipeline rate (so Eq. 3 gives th_max).  Ratios
    are measured throughput over modelled throughput, the paper's convention (Section 6.2)."""
    tun = plan.tuning
    k = 1 if tun["variant"] == 1 else tun["k"]
    gm = plan.model(T)
    nx, ny, nz = dims
    eq = S.stencil_model_estimate(ndim=ndim, rad=rad, par_vec=16384, par_time=k, f_max_hz=2.4e9, size_cell=4,
                                  num_read=nread, num_write=1, bsize_x=bsize[0], bsize_y=bsize[1], dim_x=nx,
                                  dim_y=ny, dim_z=nz, iter=T, th_max_gbs=HBM_PEAK_GBS)
    cells = nx * ny * nz
    meas_gbs = (nread + 1) * 4.0 * cells * T / (ms * 1e-3) / 1e9
    return {"k": k, "measured_ms": round(ms, 3), "model_ms": round(gm["seconds"] * 1e3, 3),
            "model_mem_ms": round(gm["mem_seconds"] * 1e3, 3), "model_alu_ms": round(gm["alu_seconds"] * 1e3, 3),
            "measured_over_model": round(gm["seconds"] * 1e3 / ms, 3),
            "eq9_gbs": round(eq["throughput_gbs"], 1), "measured_gbs_eq9": round(meas_gbs, 1),
            "measured_over_eq9": round(meas_gbs / eq["throughput_gbs"], 3)}


def tb2d_symbol(K, hot, full, split, phys=False, depth=None):
    if depth is None:
        depth = 4 if (not hot) or (hot and split and 8 < K <= 12) else 2
    return "tb2d_kernel<%d, 4, %s, false, false, %s, %d, %s, %s>" % (
        K, "true" if hot else "false", "true" if full else "false", depth, "true" if split else "false",
        "true" if phys else "false")


def tb3d_symbol(K, hot, adj, acc, full):
    if adj:
        R, NW = 2, 16
    else:
        R = 3 if (K <= 3 if hot else K <= 4) else 6
        NW = 48 // R
    b = lambda v: "true" if v else "false"
    return "tb3d_kernel<%d, 2, %d, %d, %s, %s, %s, %s, 1>" % (K, R, NW, b(hot), b(adj), b(acc), b(full))


# ------------------------------------------------------------------ CPU baseline

def host_facts():
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    llc = None
    for idx in (3, 2):
        try:
            with open("/sys/devices/system/cpu/cpu0/cache/index%d/size" % idx) as fh:
                llc = fh.read().strip()
            break
        except OSError:
            continue
    try:
        affinity = len(os.sched_getaffinity(0))
    except AttributeError:
        affinity = None
    return {"cpu_model": model, "nproc": os.cpu_count(), "affinity_cpus": affinity, "llc_per_core_group": llc}


def cpu_baseline(wl, budget_s=15.0):
    """The FP32 oracle, as it stands, on a bounded sample of the same workload: a full-width band
    of the hotspot field and power map (same coefficients) for the workload's T steps, or fewer
    if they would take more than about `budget_s` seconds.  The band's working set (field, next
    field, source and power, 4 x 512 MiB) is far beyond the host's last-level cache, as the full
    grid's is.  The rate is measured after two warm-up steps (first touch of the buffers)."""
    import oracle
    rows = 8192
    x0 = np.ascontiguousarray(wl.field()[:rows])
    p = np.ascontiguousarray(wl.power()[:rows])
    oracle.forward(x0, wl.coeffs, 2, power=p, dtype=np.float32)
    t0 = time.perf_counter()
    oracle.forward(x0, wl.coeffs, 8, power=p, dtype=np.float32)
    per_step = max((time.perf_counter() - t0) / 8, 1e-6)
    steps = max(8, min(wl.T, int(budget_s / per_step)))
    t0 = time.perf_counter()
    oracle.forward(x0, wl.coeffs, steps, power=p, dtype=np.float32)
    dt = time.perf_counter() - t0
    cells = x0.size
    out = {"value": round(cells * steps / dt / 1e9, 4), "unit": "GCell/s", "cores": oracle.num_threads(),
           "kind": "oracle",
           "sample": "FP32 oracle, hotspot 2D full-width band %d x %d of the same field and power, %d steps, %.1f s; "
                     "working set %d MiB (beyond the last-level cache)" % (
                         rows, x0.shape[1], steps, dt, 4 * cells * 4 // 2 ** 20)}
    out.update(host_facts())
    return out


# ------------------------------------------------------------------ workloads

def main_workload(S, args, dev, stream, copy_gbs):
    import torch
    from workloads import WORKLOADS, HOTSPOT
    wl = WORKLOADS["hotspot2d_16384"]
    log("[bench] generating %s inputs" % wl.name)
    x = torch.from_numpy(wl.field()).to(dev)
    p = torch.from_numpy(wl.power()).to(dev)
    if args.copy_calib:
        dst = torch.empty_like(x)
        for _ in range(3):
            dst.copy_(x)
        torch.cuda.synchronize()
        log("[bench] copy calibration: 3 copies of %d bytes" % (x.numel() * 4))
        del dst
    if args.k > 0:
        plan = S.Plan(HOTSPOT, wl.shape, {"variant": 2, "k": args.k, "seg_len": args.seg})
    else:
        plan = S.Plan(HOTSPOT, wl.shape)
    tun = plan.tuning
    log("[bench] tuning %s" % tun)
    cf = wl.coeffs

    def step():
        plan.run(x, cf, wl.T, p)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record(stream)
    for _ in range(args.steps):
        step()
    e1.record(stream)
    e1.synchronize()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = e0.elapsed_time(e1) / args.steps
    gcells = wl.cells * wl.T / (ms * 1e-3) / 1e9
    log("[bench] main: %.3f ms per run, %.1f GCell/s (wall %.2f s)" % (ms, gcells, wall))

    # Dominant kernel: the full K-step pass.  A run is T // K full passes plus, when K does not
    # divide T, one shorter pass (on a smaller instantiation) and, for an odd pass count, a
    # parity copy; both are timed on their own with the same events and taken out, and the
    # full passes' average launch duration is what remains divided by their number.  A split
    # pass runs the edge-free kernel (about 95% of the tiles, the whole pass long) while the
    # frame kernel runs beside it on a second stream, so the pass time bounds its duration.
    K, seg = tun["k"], tun["seg_len"]
    n_full, rem = divmod(wl.T, K)
    passes = n_full + (1 if rem else 0)
    tmp = torch.empty_like(x)
    cp_ms = time_call(lambda: tmp.copy_(x), stream, 5)
    del tmp
    short_ms = 0.0
    if rem:
        short_ms = max(0.0, time_call(lambda: plan.run(x, cf, rem, p), stream, 5) - cp_ms)
    kern_ms = (ms - (cp_ms if passes % 2 == 1 else 0.0) - short_ms) / n_full
    split = tb2d_split(wl.nx, wl.ny, K, K, seg)
    b, f = tb2d_pass(wl.nx, wl.ny, K, K, seg, 2, 10, interior_only=split)
    roof = roofline(tb2d_symbol(K, True, True, split), "tb2d_hot", {"k": K, "seg_len": seg, "shape": list(wl.shape)},
                    kern_ms, b, f, copy_gbs)
    roof["launches_per_run"] = n_full
    study = model_row(S, plan, wl.T, ms, 2, 2, (wl.nx, wl.ny, 1), (256, 0))
    plan.close()
    return x, p, ms, gcells, tun, roof, study


def plain_hotspot2d(S, x, p, stream, copy_gbs):
    from workloads import WORKLOADS, HOTSPOT
    wl = WORKLOADS["hotspot2d_16384"]
    pl = S.Plan(HOTSPOT, wl.shape, {"variant": 1})
    Tp = 100
    pl.run(x, wl.coeffs, 4, p)
    ms = time_call(lambda: pl.run(x, wl.coeffs, Tp, p), stream, 2)
    g = wl.cells * Tp / (ms * 1e-3) / 1e9
    # one launch per step: reads the field and the power map, writes the field (Table 2: 12 B);
    # 12 FLOP per update as executed (the source FMA and five FMAs)
    roof = roofline("plain_kernel<true, false, false, false>", "plain", {"shape": list(wl.shape)}, ms / Tp,
                    12.0 * wl.cells, 12.0 * wl.cells, copy_gbs)
    study = model_row(S, pl, Tp, ms, 2, 2, (wl.nx, wl.ny, 1), (wl.nx + 2, 0))
    pl.close()
    return {"gcells": round(g, 1), "ms_per_step_update": round(ms / Tp, 4), "hbm_gbs_eff": round(g * 12, 1),
            "roofline": roof}, study


def phys2d(S, dev, stream, copy_gbs):
    import torch
    from workloads import WORKLOADS
    w6 = WORKLOADS["hotspot2d_phys_16384"]
    x6 = torch.from_numpy(w6.field()).to(dev)
    p6 = torch.from_numpy(w6.power()).to(dev)
    pl6 = S.Plan(S.HOTSPOT_PHYS, w6.shape)
    pl6.run(x6, w6.coeffs, 24, p6)
    ms6 = time_call(lambda: pl6.run(x6, w6.coeffs, w6.T, p6), stream, 2)
    g6 = w6.cells * w6.T / (ms6 * 1e-3) / 1e9
    t6 = pl6.tuning
    K, seg = t6["k"], t6["seg_len"]
    # per launch: 8 full passes (an even count, no parity copy)
    lms = time_call(lambda: pl6.run(x6, w6.coeffs, 8 * K, p6), stream, 2) / 8
    split = tb2d_split(w6.nx, w6.ny, K, K, seg)
    # Table 2's 15 FLOP per cell update: 2 adds, 2 FMAs for the differences, 1 subtraction, 4 FMAs
    b, f = tb2d_pass(w6.nx, w6.ny, K, K, seg, 2, 15, interior_only=split)
    roof = roofline(tb2d_symbol(K, True, True, split, phys=True), "tb2d_phys",
                    {"k": K, "seg_len": seg, "shape": list(w6.shape)}, lms, b, f, copy_gbs)
    study = model_row(S, pl6, w6.T, ms6, 2, 2, (w6.nx, w6.ny, 1), (256, 0))
    pl6.close()
    return {"gcells": round(g6, 1), "ms_per_run": round(ms6, 2), "k": K, "seg_len": seg,
            "pct_single_pass_roofline": round(100 * g6 / (HBM_PEAK_GBS / 12), 1), "roofline": roof}, study


def star2d(S, args, dev, stream, copy_gbs):
    import torch
    from workloads import STAR_WORKLOAD, STAR_SETS, star_field
    w7 = STAR_WORKLOAD
    x7 = torch.from_numpy(star_field(w7)).to(dev)
    pl7 = S.StarPlan(w7["rad"], (w7["ny"], w7["nx"]),
                     {"variant": 2, "k": args.star_k, "seg_len": args.star_seg} if args.star_k > 0 else None)
    wt7 = STAR_SETS[w7["rad"]]
    pl7.run(x7, wt7, 16)
    ms7 = time_call(lambda: pl7.run(x7, wt7, w7["T"]), stream, 2)
    c7 = w7["nx"] * w7["ny"]
    g7 = c7 * w7["T"] / (ms7 * 1e-3) / 1e9
    t7 = pl7.tuning
    K, seg, R = t7["k"], t7["seg_len"], w7["rad"]
    lms = time_call(lambda: pl7.run(x7, wt7, 8 * K), stream, 2) / 8
    # a multiply and 4r FMAs per cell update: 8r + 1 FLOP
    b, f = tb2d_pass(w7["nx"], w7["ny"], K, K, seg, 1, 8 * R + 1, R=R)
    roof = roofline("star2d_kernel<%d, %d, true, false>" % (R, K), "star2d", {"k": K, "seg_len": seg, "rad": R}, lms, b, f,
                    copy_gbs)
    pp7 = S.StarPlan(w7["rad"], (w7["ny"], w7["nx"]), {"variant": 1})
    msp7 = time_call(lambda: pp7.run(x7, wt7, 20), stream, 1)
    gp7 = c7 * 20 / (msp7 * 1e-3) / 1e9
    study = model_row(S, pl7, w7["T"], ms7, 2, 1, (w7["nx"], w7["ny"], 1), (256, 0), rad=R)
    pl7.close()
    pp7.close()
    return {"gcells": round(g7, 1), "ms_per_run": round(ms7, 2), "k": K, "seg_len": seg,
            "gcells_one_step": round(gp7, 1), "pct_single_pass_roofline": round(100 * g7 / (HBM_PEAK_GBS / 8), 1),
            "roofline": roof}, study


def star3d(S, dev, stream, copy_gbs):
    import torch
    from workloads import STAR3_WORKLOAD, STAR3_SETS, star3_field
    w = STAR3_WORKLOAD
    x = torch.from_numpy(star3_field(w)).to(dev)
    shape = (w["nz"], w["ny"], w["nx"])
    R, T = w["rad"], w["T"]
    pl = S.StarPlan(R, shape)
    wt = STAR3_SETS[R]
    pl.run(x, wt, 4)
    ms = time_call(lambda: pl.run(x, wt, T), stream, 2)
    cells = w["nx"] * w["ny"] * w["nz"]
    g = cells * T / (ms * 1e-3) / 1e9
    t = pl.tuning
    K, seg = t["k"], t["seg_len"]
    lms = time_call(lambda: pl.run(x, wt, 8 * K), stream, 2) / 8
    b, f = star3d_pass(w["nx"], w["ny"], w["nz"], R, K, seg)
    roof = roofline("star3d_kernel<%d, %d, false>" % (R, K), "star3d", {"k": K, "seg_len": seg, "rad": R}, lms, b, f,
                    copy_gbs)
    pp = S.StarPlan(R, shape, {"variant": 1})
    pp.run(x, wt, 2)
    msp = time_call(lambda: pp.run(x, wt, 20), stream, 1)
    gp = cells * 20 / (msp * 1e-3) / 1e9
    # the adjoint sweep: one transposed step per launch, reading lambda (neighbours from L1/L2)
    # and writing it once: 8 B per cell and step; 12R + 1 FLOP per cell (interior cells)
    gx = torch.empty_like(x)
    pl.adjoint(x, wt, 2, gx)
    msa = time_call(lambda: pl.adjoint(x, wt, 20, gx), stream, 2) / 20
    roof_a = roofline("star_adjoint_v4_kernel<3, %d>" % R, "star_adj", {"rad": R, "shape": list(shape)}, msa, 8.0 * cells,
                      (12 * R + 1) * float(cells), copy_gbs)
    study = model_row(S, pl, T, ms, 3, 1, (w["nx"], w["ny"], w["nz"]), (64, 64), rad=R)
    pl.close()
    pp.close()
    return {"gcells": round(g, 1), "ms_per_run": round(ms, 2), "k": K, "seg_len": seg,
            "gcells_one_step": round(gp, 1), "speedup_vs_one_step": round(g / gp, 2),
            "gcells_adjoint": round(cells / (msa * 1e-3) / 1e9, 1),
            "pct_single_pass_roofline": round(100 * g / (HBM_PEAK_GBS / 8), 1), "roofline": roof,
            "roofline_adjoint": roof_a}, study


def diffusion3d(S, dev, stream, copy_gbs):
    import torch
    from workloads import WORKLOADS, DIFFUSION
    w3 = WORKLOADS["diffusion3d_512"]
    x3 = torch.from_numpy(w3.field()).to(dev)
    pl3 = S.Plan(DIFFUSION, w3.shape)
    pl3.run(x3, w3.coeffs, 8)
    ms3 = time_call(lambda: pl3.run(x3, w3.coeffs, w3.T), stream, 2)
    g3 = w3.cells * w3.T / (ms3 * 1e-3) / 1e9
    t3 = pl3.tuning
    K = t3["k"]
    lms = time_call(lambda: pl3.run(x3, w3.coeffs, 8 * K), stream, 2) / 8
    # 13 FLOP per cell and level as executed: a multiply and six FMAs
    b, f = tb3d_pass(w3.nx, w3.ny, w3.nz, K, K, t3, 1, 4, 13)
    roof = roofline(tb3d_symbol(K, False, False, False, True), "tb3d_diff",
                    {"k": K, "nwork": t3["nwork"], "seg_len": t3["seg_len"], "shape": list(w3.shape)}, lms, b, f,
                    copy_gbs)
    pp3 = S.Plan(DIFFUSION, w3.shape, {"variant": 1})
    pp3.run(x3, w3.coeffs, 2)
    msp3 = time_call(lambda: pp3.run(x3, w3.coeffs, 40), stream, 1)
    gp3 = w3.cells * 40 / (msp3 * 1e-3) / 1e9
    roof_p = roofline("plain_kernel<false, false, false, false>", "plain", {"shape": list(w3.shape)}, msp3 / 40,
                      8.0 * w3.cells, 13.0 * w3.cells, copy_gbs)
    study = model_row(S, pl3, w3.T, ms3, 3, 1, (w3.nx, w3.ny, w3.nz), (t3["bsize_x"], t3["bsize_y"]))
    pl3.close()
    pp3.close()
    return {"gcells_tb": round(g3, 1), "ms_tb": round(ms3, 2), "k": K, "nwork": t3["nwork"],
            "gcells_plain": round(gp3, 1), "speedup_tb_vs_plain": round(g3 / gp3, 2),
            "pct_single_pass_roofline": round(100 * g3 / (HBM_PEAK_GBS / 8), 1),
            "roofline": roof, "roofline_plain": roof_p}, study


def diffusion2d_small(S, dev, stream, copy_gbs):
    import torch
    from workloads import WORKLOADS, DIFFUSION
    w1 = WORKLOADS["diffusion2d_256"]
    x1 = torch.from_numpy(w1.field()).to(dev)
    pl1 = S.Plan(DIFFUSION, w1.shape)
    pl1.run(x1, w1.coeffs, w1.T)
    ms1 = time_call(lambda: pl1.run(x1, w1.coeffs, w1.T), stream, 20)
    t1 = pl1.tuning
    K, seg = t1["k"], t1["seg_len"]
    lms = time_call(lambda: pl1.run(x1, w1.coeffs, 8 * K), stream, 10) / 8
    b, f = tb2d_pass(w1.nx, w1.ny, K, K, seg, 1, 9)
    roof = roofline(tb2d_symbol(K, False, True, False), "tb2d_diff", {"k": K, "seg_len": seg}, lms, b, f, copy_gbs,
                    note="256^2 grid: a pass is a handful of tiles, launch and latency bound")
    study = model_row(S, pl1, w1.T, ms1, 2, 1, (w1.nx, w1.ny, 1), (256, 0))
    pl1.close()
    return {"us_per_run": round(ms1 * 1e3, 1), "gcells": round(w1.cells * w1.T / (ms1 * 1e-3) / 1e9, 1),
            "k": K, "roofline": roof}, study


def hotspot3d(S, dev, stream, copy_gbs):
    """Forward with checkpoints, adjoint and adjoint with verified recompute, each warmed up and
    timed over several calls with HIP events (the first run_ckpt allocates the checkpoints)."""
    import torch
    from workloads import WORKLOADS, HOTSPOT
    w5 = WORKLOADS["hotspot3d_256_adjoint"]
    x5 = torch.from_numpy(w5.field()).to(dev)
    p5 = torch.from_numpy(w5.power()).to(dev)
    y5 = torch.from_numpy(w5.target()).to(dev)
    pl5 = S.Plan(HOTSPOT, w5.shape)
    xs = x5.clone()
    pl5.run_ckpt(xs, w5.coeffs, w5.T, w5.ckpt_every, p5)  # warm-up: allocates the checkpoints
    fwd_ms = time_call(lambda: pl5.run_ckpt(xs, w5.coeffs, w5.T, w5.ckpt_every, p5), stream, 3)
    xs.copy_(x5)
    pl5.run_ckpt(xs, w5.coeffs, w5.T, w5.ckpt_every, p5)
    cot = (xs - y5).contiguous()
    gx = torch.empty_like(x5)
    gp = torch.empty_like(x5)
    pl5.adjoint(cot, w5.coeffs, w5.T, gx, gp, p5, 0)
    adj_ms = time_call(lambda: pl5.adjoint(cot, w5.coeffs, w5.T, gx, gp, p5, 0), stream, 3)
    pl5.adjoint(cot, w5.coeffs, w5.T, gx, gp, p5, 1)  # warm-up: allocates the check buffer
    rc_ms = time_call(lambda: pl5.adjoint(cot, w5.coeffs, w5.T, gx, gp, p5, 1), stream, 2)
    t5 = pl5.tuning
    ta = pl5.adjoint_tuning
    K, KA = t5["k"], ta["k"]
    lms = time_call(lambda: pl5.run(xs, w5.coeffs, 8 * K, p5), stream, 2) / 8
    lams = time_call(lambda: pl5.adjoint(cot, w5.coeffs, 8 * KA, gx, gp, None, 0), stream, 2) / 8
    # forward: 15 FLOP per cell and level as executed (the source FMA, the centre FMA, six FMAs);
    # the power plane is read once per pass (the kernel re-reads it from L2 at every level)
    b, f = tb3d_pass(w5.nx, w5.ny, w5.nz, K, K, t5, 2, 4, 16)
    roof = roofline(tb3d_symbol(K, True, False, False, True), "tb3d_hot",
                    {"k": K, "nwork": t5["nwork"], "seg_len": t5["seg_len"], "shape": list(w5.shape)}, lms, b, f,
                    copy_gbs)
    # adjoint: reads the lambda window, writes lambda and reads and writes grad_p (12 B per cell);
    # 13 FLOP per cell and level plus the running sum
    ba, fa = tb3d_pass(w5.nx, w5.ny, w5.nz, KA, KA, ta, 1, 12, 14)
    roof_a = roofline(tb3d_symbol(KA, False, True, True, True), "tb3d_adj",
                      {"k": KA, "nwork": ta["nwork"], "seg_len": ta["seg_len"], "shape": list(w5.shape)}, lams, ba,
                      fa, copy_gbs)
    study = model_row(S, pl5, w5.T, fwd_ms, 3, 2, (w5.nx, w5.ny, w5.nz), (t5["bsize_x"], t5["bsize_y"]))
    pl5.close()
    return {"fwd_ckpt_ms": round(fwd_ms, 2), "adjoint_ms": round(adj_ms, 2), "adjoint_recompute_ms": round(rc_ms, 2),
            "ratio_adjoint_fwd": round(adj_ms / fwd_ms, 2), "ratio_recompute_fwd": round(rc_ms / fwd_ms, 2),
            "gcells_fwd": round(w5.cells * w5.T / (fwd_ms * 1e-3) / 1e9, 1), "k": K, "k_adjoint": KA,
            "roofline": roof, "roofline_adjoint": roof_a}, study


def batched(S, dev, stream, copy_gbs):
    import torch
    from workloads import SETS, batch_grids
    grids = batch_grids()
    xs = [torch.from_numpy(g.field()).to(dev) for g in grids]
    cfs = [SETS[g.coef_set] for g in grids]
    ts = [g.T for g in grids]
    cache = S.run_batched(xs, cfs, ts)
    torch.cuda.synchronize()
    bms = time_call(lambda: S.run_batched(xs, cfs, ts, cache=cache), stream, 2)
    S.stencil_batch_sync(cache)
    S.stencil_batch_destroy(cache)
    upd = sum(g.cells * g.T for g in grids)
    out = {"ms": round(bms, 2), "updates": upd, "gcells_aggregate": round(upd / (bms * 1e-3) / 1e9, 1)}
    # each persistent kernel on its own: the batch of the 2D grids, then of the 3D grids
    for nd, cap, sym, fl in ((2, 16, "batched2d_kernel(BLaunch)", 9), (3, 4, "batched3d_kernel(BLaunch)", 13)):
        idx = [i for i, g in enumerate(grids) if g.ndim == nd]
        sx, sc, st = [xs[i] for i in idx], [cfs[i] for i in idx], [ts[i] for i in idx]
        c = S.run_batched(sx, sc, st)
        torch.cuda.synchronize()
        kms = time_call(lambda: S.run_batched(sx, sc, st, cache=c), stream, 2)
        S.stencil_batch_destroy(c)
        # each grid runs an even number of passes of at most `cap` steps; per pass every cell is
        # read and written once (the halo rows that overlapping windows read again are not
        # counted, so this is a lower bound of the algorithmic bytes), and every update executes
        # `fl` FLOP at least (halo cells are not counted either)
        passes = [max(2, 2 * math.ceil(math.ceil(grids[i].T / cap) / 2)) if grids[i].T > 0 else 0 for i in idx]
        bytes_ = sum(8.0 * grids[i].cells * n for i, n in zip(idx, passes))
        flops = sum(float(fl) * grids[i].cells * grids[i].T for i in idx)
        u = sum(grids[i].cells * grids[i].T for i in idx)
        out["roofline_%dd" % nd] = roofline(sym, "batched", {"grids": len(idx)}, kms, bytes_, flops, copy_gbs,
                                            note="one launch = the whole %dD half of the batch (graph replay); bytes "
                                                 "and FLOPs are lower bounds (halos not counted)" % nd)
        out["gcells_%dd" % nd] = round(u / (kms * 1e-3) / 1e9, 1)
    del xs
    return out


def slab3d(S, dev, stream, copy_gbs):
    """One device's share of a 512^3 grid cut into slabs along z: 64 interior planes with 4
    ghost planes per face, one pass of 4 fused steps."""
    import torch
    from workloads import SETS, DIFFUSION, uniform
    k, nz_in, g = 4, 64, 4
    shape = (nz_in + 2 * g, 512, 512)
    src = torch.from_numpy(uniform(shape, 0.0, 1.0, 9400)).to(dev)
    dst = torch.empty_like(src)
    pl = S.Plan(DIFFUSION, shape, {"variant": 2, "k": k})
    cf = SETS["D3"]
    pl.run_slab(src, dst, cf, k, g, g)
    ms = time_call(lambda: pl.run_slab(src, dst, cf, k, g, g), stream, 20)
    t = pl.tuning
    b, f = tb3d_pass(512, 512, shape[0], k, k, t, 1, 4, 13, zlo=g, zhi=shape[0] - g)
    roof = roofline(tb3d_symbol(k, False, False, False, True), "tb3d_diff",
                    {"k": k, "nwork": t["nwork"], "seg_len": t["seg_len"], "shape": list(shape)}, ms, b, f, copy_gbs)
    pl.close()
    upd = 512 * 512 * nz_in * k
    return {"ms_per_pass": round(ms, 4), "gcells_interior": round(upd / (ms * 1e-3) / 1e9, 1), "k": k,
            "roofline": roof}


# ------------------------------------------------------------------ main

def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--quick", action="store_true", help="main workload only")
    ap.add_argument("--only", default="", help="comma-separated secondary workloads to run (default: all)")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--k", type=int, default=0, help="fix the fused steps per pass (skips auto-tuning)")
    ap.add_argument("--seg", type=int, default=0, help="fix the rows per tile pass (with --k)")
    ap.add_argument("--star-k", type=int, default=0,
                    help="fix the fused steps per pass of the radius-2 star workload (skips its tuning)")
    ap.add_argument("--star-seg", type=int, default=0, help="fix its rows per tile pass (with --star-k)")
    ap.add_argument("--copy-calib", action="store_true",
                    help="first copy one grid-sized buffer three times (a known-size kernel for "
                         "calibrating memory counters)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU only: this library has no multi-GPU path (the slab pass is one "
              "device's share; the exchange over xGMI is design-only).", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_1802_00438_amd as S
    from workloads import WORKLOADS

    assert torch.cuda.is_available(), "bench needs a GPU"
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream()
    wl = WORKLOADS["hotspot2d_16384"]

    # copy bandwidth of this device: the achievable ceiling beside the 8 TB/s peak
    probe = torch.empty(wl.shape, dtype=torch.float32, device=dev).fill_(1.0)
    copy_gbs, copy_ms = copy_bandwidth(probe, stream)
    del probe
    log("[bench] copy bandwidth %.1f GB/s" % copy_gbs)

    x, p, ms, gcells, tun, roof, study0 = main_workload(S, args, dev, stream, copy_gbs)
    out = {
        "metric": "GCell-updates/s & % HBM roofline (fwd, adjoint) vs plain 1-step/pass kernel",
        "value": round(gcells, 2),
        "unit": "GCell/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "hotspot2d_16384", "nx": wl.nx, "ny": wl.ny, "T": wl.T, "coeffs": "H2",
                   "k": tun["k"], "seg_len": tun["seg_len"], "bsize_x": tun["bsize_x"]},
        "pct_single_pass_roofline": round(100.0 * gcells / (HBM_PEAK_GBS / 12.0), 1),
        "effective_gbs_eq9": round(gcells * 12.0, 1),
        "effective_gflops_table2": round(gcells * 15.0, 1),
        "roofline": roof,
        "copy_bw": {"gbs": round(copy_gbs, 1), "frac_of_peak": round(copy_gbs / HBM_PEAK_GBS, 4),
                    "method": "device-to-device copy of a 1 GiB tensor, read + write bytes over its time "
                              "(HIP events, 5 copies after a warm-up)"},
        # context only (another machine and stencil): the paper's headline results, Diffusion 2D
        # and 3D on an Arria 10 GX 1150 FPGA (Section 6, abstract)
        "paper_context_gflops": {"diffusion2d_arria10": 758.2, "diffusion3d_arria10": 374.7},
    }
    extras, study = {}, {"hotspot2d_16384": study0}
    only = [w for w in args.only.split(",") if w] or SECONDARY
    unknown = [w for w in only if w not in SECONDARY]
    if unknown:
        log("[bench] unknown workloads %s (choose from %s)" % (unknown, SECONDARY))
        sys.exit(2)
    if not args.quick:
        if "plain_hotspot2d_16384" in only:
            extras["plain_hotspot2d_16384"], study["plain_hotspot2d_16384"] = plain_hotspot2d(S, x, p, stream,
                                                                                              copy_gbs)
            extras["plain_hotspot2d_16384"]["speedup_tb_vs_plain"] = round(
                gcells / extras["plain_hotspot2d_16384"]["gcells"], 2)
            log("[bench] plain hotspot 2D: %.1f GCell/s" % extras["plain_hotspot2d_16384"]["gcells"])
    del x, p
    torch.cuda.empty_cache()
    runners = [("hotspot2d_phys_16384", lambda: phys2d(S, dev, stream, copy_gbs)),
               ("star2d_r2_16384", lambda: star2d(S, args, dev, stream, copy_gbs)),
               ("star3d_r2_512", lambda: star3d(S, dev, stream, copy_gbs)),
               ("diffusion3d_512", lambda: diffusion3d(S, dev, stream, copy_gbs)),
               ("diffusion2d_256", lambda: diffusion2d_small(S, dev, stream, copy_gbs)),
               ("hotspot3d_256", lambda: hotspot3d(S, dev, stream, copy_gbs)),
               ("batched_64", lambda: (batched(S, dev, stream, copy_gbs), None)),
               ("slab3d_512x512x64", lambda: (slab3d(S, dev, stream, copy_gbs), None))]
    if not args.quick:
        for name, fn in runners:
            if name not in only:
                continue
            res, row = fn()
            extras[name] = res
            if row is not None:
                study[name] = row
            torch.cuda.empty_cache()
            log("[bench] %s: %s" % (name, {k: v for k, v in res.items() if not k.startswith("roofline")}))
    out["other_workloads"] = extras
    out["model_accuracy"] = study
    if not args.no_cpu:
        log("[bench] CPU oracle baseline")
        out["cpu_baseline"] = cpu_baseline(wl)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
