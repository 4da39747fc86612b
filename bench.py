"""Benchmark: temporal-blocked hotspot 2D, 16384 x 16384 cells, 1000 time steps, one MI355X.

One "step" of this bench is one whole run of the hot path: stencil_run over the 16384^2
hotspot grid for T = 1000 time steps (all passes, boundary handling, ping-pong), with the
temperature and power maps already resident in HBM.  value = cell updates per second
(GCell/s); the single-pass HBM roofline of this stencil is 8 TB/s / 12 B = 667 GCell/s
(Table 2 bytes per update).  The same JSON line carries, for the dominant kernel, the
achieved rate against its roofline, the CPU oracle timed on a bounded sample, and (unless
--quick) the plain one-step-per-launch kernel, the 3D and batched workloads and the adjoint.
`model_accuracy` sets each measured workload against the library's own time model and the
paper's Eq. 3-9 model at the same blocking (measured over modelled throughput).

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--quick]
"""
import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz x 2 FLOP per FMA, plain (non-packed) FP32
ALU_PEAK_TFLOPS = 256 * 4 * 16 * 2.4e9 * 2 / 1e12


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def tb2d_geometry(nx, ny, K, seg):
    """Tile geometry of a temporal-blocked 2D pass: 256-column windows with a left halo kr
    (K rounded up to 4) and cs output columns, by `seg`-row segments."""
    W = 256
    kr = (K + 3) // 4 * 4
    cs = (W - K - kr) // 4 * 4
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


def tb2d_bytes_flops(nx, ny, K, keff, seg, hot=True, interior_only=False):
    """Algorithmic HBM bytes and executed FP32 FLOPs of one temporal-blocked 2D pass with
    keff fused steps (or of its interior tiles only): every window row of a tile is read once
    per pass (temperature, plus power for hotspot) and every output cell is written once."""
    W, kr, cs, ntx, seg, nseg = tb2d_geometry(nx, ny, K, seg)
    if interior_only:
        xs, ys = tb2d_interior(nx, ny, K, keff, seg)
    else:
        xs, ys = list(range(ntx)), list(range(nseg))
    tiles = len(xs) * len(ys)
    out_cells = sum(min(cs, nx - tx * cs) for tx in xs) * sum(min(seg, ny - sg * seg) for sg in ys)
    rows = seg + 2 * keff
    nread = 2 if hot else 1
    bytes_ = tiles * rows * W * 4 * nread + out_cells * 4
    # per cell and level: hotspot fma(cc, c, q) + 4 fma; diffusion mul + 4 fma (FMA = 2 FLOP)
    flops_per = 10 if hot else 9
    flops = tiles * W * (seg + keff) * keff * flops_per
    return bytes_, flops


def run_roofline(nx, ny, T, k, kinst, seg, R, nread, flops_per, ms):
    """Whole-run rates of a temporal-blocked 2D workload against both roofs: algorithmic HBM
    bytes (each tile's window rows read once per pass, nread fields, one write per cell) and
    executed FLOPs (flops_per per computed cell and level, halos included) summed over the
    passes of T steps (full passes of k steps, then one of T mod k on the smallest instantiated
    K that holds it), over the measured run time in ms."""
    def one(K, keff):
        W = 256
        kr = (R * K + 3) // 4 * 4
        cs = (W - R * K - kr) // 4 * 4
        sg = max(1, min(seg, ny))
        tiles = math.ceil(nx / cs) * math.ceil(ny / sg)
        b = tiles * (sg + 2 * R * keff) * W * 4 * nread + nx * ny * 4
        f = tiles * W * (sg + R * keff) * keff * flops_per
        return b, f
    nfull, rem = divmod(T, k)
    b, f = one(kinst(k), k)
    B, F = nfull * b, nfull * f
    if rem:
        b, f = one(kinst(rem), rem)
        B, F = B + b, F + f
    gbs = B / (ms * 1e-3) / 1e9
    tf = F / (ms * 1e-3) / 1e12
    fh, fa = gbs / HBM_PEAK_GBS, tf / ALU_PEAK_TFLOPS
    if fa >= fh:
        r = {"bound": "alu", "achieved": round(tf, 3), "peak": round(ALU_PEAK_TFLOPS, 1), "unit": "TFLOP/s", "frac": round(fa, 4)}
    else:
        r = {"bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(fh, 4)}
    r.update({"frac_alu": round(fa, 4), "frac_hbm": round(fh, 4), "scope": "whole run (all passes and kernels)"})
    return r


def smallest_at_least(ks):
    return lambda k: min([K for K in ks if K >= k] or [max(ks)])


# Kernel sources whose hash identifies the measured build of the dominant kernel.
TB2D_SOURCES = ["tb2d.hpp", "device_common.hpp", "k_tb2d_hot.hip"]
PMC_SUMMARY = os.path.join(ROOT, "profiles", "tb2d_hotspot_16384_hbm_counters.md")


def kernel_source_hash():
    import hashlib
    h = hashlib.sha256()
    for f in TB2D_SOURCES:
        with open(os.path.join(ROOT, "paper_1802_00438_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(K, seg):
    """HBM bytes per launch of the dominant kernel from the committed counter summary
    (FETCH_SIZE and WRITE_SIZE per dispatch, each divided by what the counter reads per byte
    of a plain device copy), or None if the summary is missing or was taken on another
    kernel build or tile configuration."""
    try:
        with open(PMC_SUMMARY) as fh:
            text = fh.read()
        blob = text.split("<!-- counters-json -->")[1].split("<!-- /counters-json -->")[0]
        rec = json.loads(blob.strip().strip("`").strip())
    except (OSError, IndexError, ValueError):
        return None
    if rec.get("source_hash") != kernel_source_hash() or rec.get("k") != K or rec.get("seg_len") != seg:
        return None
    return (rec["fetch_kib_per_dispatch"] * 1024.0 / rec["copy_fetch_factor"] +
            rec["write_kib_per_dispatch"] * 1024.0 / rec["copy_write_factor"])


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


def time_call(fn, stream, reps):
    import torch
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(reps):
        fn()
    e1.record(stream)
    e1.synchronize()
    return e0.elapsed_time(e1) / reps


def cpu_baseline(wl, budget_s=12.0):
    """The FP32 oracle on a bounded sample of the same workload (a square sub-grid of the
    hotspot field, the same coefficients), scaled to GCell/s."""
    import oracle
    side = 2048
    x0 = wl.field()[:side, :side].copy()
    p = wl.power()[:side, :side].copy()
    t0 = time.perf_counter()
    oracle.forward(x0, wl.coeffs, 4, power=p, dtype=np.float32)
    dt = max(time.perf_counter() - t0, 1e-3)
    steps = max(4, min(wl.T, int(budget_s / dt * 4)))
    t0 = time.perf_counter()
    oracle.forward(x0, wl.coeffs, steps, power=p, dtype=np.float32)
    dt = time.perf_counter() - t0
    return {"value": round(side * side * steps / dt / 1e9, 4), "unit": "GCell/s", "cores": oracle.num_threads(),
            "kind": "oracle",
            "sample": "FP32 oracle, hotspot 2D %dx%d sub-grid of the same field, %d steps, %.1f s" % (
                side, side, steps, dt)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--quick", action="store_true", help="main workload only")
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
        print("bench.py measures one GPU only: this library has no multi-GPU path (the slab "
              "decomposition over xGMI is design-only).", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_1802_00438_amd as S
    from workloads import WORKLOADS, SETS, HOTSPOT, DIFFUSION, batch_grids

    assert torch.cuda.is_available(), "bench needs a GPU"
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream()
    wl = WORKLOADS["hotspot2d_16384"]
    cells = wl.cells
    log("[bench] generating %s inputs" % wl.name)
    x_host = wl.field()
    p_host = wl.power()
    x = torch.from_numpy(x_host).to(dev)
    p = torch.from_numpy(p_host).to(dev)
    del x_host
    if args.copy_calib:
        dst = torch.empty_like(x)
        for _ in range(3):
            dst.copy_(x)
        torch.cuda.synchronize()
        log("[bench] copy calibration: 3 copies of %d bytes" % (x.numel() * 4))
        del dst
    if args.k > 0:
        log("[bench] creating plan (k=%d, seg=%d)" % (args.k, args.seg))
        plan = S.Plan(HOTSPOT, wl.shape, {"variant": 2, "k": args.k, "seg_len": args.seg})
    else:
        log("[bench] creating plan (auto-tune)")
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
    for i in range(args.steps):
        step()
    e1.record(stream)
    e1.synchronize()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = e0.elapsed_time(e1) / args.steps
    gcells = cells * wl.T / (ms * 1e-3) / 1e9
    log("[bench] main: %.3f ms per run, %.1f GCell/s (wall %.2f s)" % (ms, gcells, wall))

    # Dominant kernel: the full K-step temporal-blocked hotspot pass.  A run is T // K full
    # passes plus, when K does not divide T, one shorter pass (on a smaller instantiation)
    # and, for an odd pass count, a parity copy.  The copy and the short pass are timed on
    # their own with the same events, and the full passes' average launch duration is what
    # remains of the timed run divided by their number.
    K = tun["k"]
    seg = tun["seg_len"]
    n_full, rem = divmod(wl.T, K)
    passes = n_full + (1 if rem else 0)
    tmp = torch.empty_like(x)
    copy_ms = time_call(lambda: tmp.copy_(x), stream, 5)
    del tmp
    short_ms = 0.0
    if rem:
        # a run of `rem` steps is one pass, preceded by the parity copy (one pass is odd)
        short_ms = max(0.0, time_call(lambda: plan.run(x, cf, rem, p), stream, 5) - copy_ms)
    kern_ms = (ms - (copy_ms if passes % 2 == 1 else 0.0) - short_ms) / n_full
    # A pass with enough interior tiles runs them in the edge-free kernel while the edge tiles
    # run beside it on a second stream; that kernel covers ~95% of the tiles and spans the
    # pass, so the pass time measured here bounds its duration from above.
    xs, ys = tb2d_interior(wl.nx, wl.ny, K, K, seg)
    split = len(xs) * len(ys) >= 1024 and len(xs) * len(ys) < tb2d_geometry(wl.nx, wl.ny, K, seg)[3] * \
        tb2d_geometry(wl.nx, wl.ny, K, seg)[5] and wl.nx % 4 == 0
    launch_bytes, launch_flops = tb2d_bytes_flops(wl.nx, wl.ny, K, K, seg, hot=True, interior_only=split)
    gbs = launch_bytes / (kern_ms * 1e-3) / 1e9
    tflops = launch_flops / (kern_ms * 1e-3) / 1e12
    frac_hbm = gbs / HBM_PEAK_GBS
    frac_alu = tflops / ALU_PEAK_TFLOPS
    traffic_bytes = measured_traffic(K, seg)
    if frac_alu >= frac_hbm:
        roof = {"bound": "alu", "achieved": round(tflops, 3), "peak": round(ALU_PEAK_TFLOPS, 1), "unit": "TFLOP/s",
                "frac": round(frac_alu, 4)}
    else:
        roof = {"bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(frac_hbm, 4)}
    # measured HBM traffic per launch over the same average launch duration, in GB/s
    roof["traffic"] = None if traffic_bytes is None else round(traffic_bytes / (kern_ms * 1e-3) / 1e9, 1)
    # the kernel symbol: four rows in flight in the edge-free hotspot kernel for 8 < K <= 12
    depth = 4 if split and 8 < K <= 12 else 2
    roof["kernel"] = "tb2d_kernel<%d, 4, true, false, false, true, %d, %s, false>" % (
        K, depth, "true" if split else "false")
    roof["avg_launch_ms"] = round(kern_ms, 4)
    roof["launches_per_run"] = n_full
    roof["algorithmic_bytes_per_launch"] = int(launch_bytes)
    roof["traffic_bytes_per_launch"] = None if traffic_bytes is None else int(traffic_bytes)
    roof["hbm_gbs_algorithmic"] = round(gbs, 1)
    roof["tflops_executed"] = round(tflops, 3)
    roof["frac_hbm"] = round(frac_hbm, 4)
    roof["frac_alu"] = round(frac_alu, 4)

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
                   "k": K, "seg_len": seg, "bsize_x": tun["bsize_x"]},
        "pct_single_pass_roofline": round(100.0 * gcells / (HBM_PEAK_GBS / 12.0), 1),
        "effective_gbs_eq9": round(gcells * 12.0, 1),
        "effective_gflops_table2": round(gcells * 15.0, 1),
        "roofline": roof,
        # context only (another machine and stencil): the paper's headline results, Diffusion 2D
        # and 3D on an Arria 10 GX 1150 FPGA (Section 6, abstract)
        "paper_context_gflops": {"diffusion2d_arria10": 758.2, "diffusion3d_arria10": 374.7},
    }

    extras = {}
    study = {}
    study["hotspot2d_16384"] = model_row(S, plan, wl.T, ms, 2, 2, (wl.nx, wl.ny, 1), (256, 0))
    if not args.quick:
        # plain one-step-per-launch comparator on the same grid (fewer steps, same per-step work)
        pplan = S.Plan(HOTSPOT, wl.shape, {"variant": 1})
        Tp = 200
        pplan.run(x, cf, 4, p)
        pms = time_call(lambda: pplan.run(x, cf, Tp, p), stream, 2)
        pg = cells * Tp / (pms * 1e-3) / 1e9
        study["plain_hotspot2d_16384"] = model_row(S, pplan, Tp, pms, 2, 2, (wl.nx, wl.ny, 1), (wl.nx + 2, 0))
        extras["plain_hotspot2d_16384"] = {"gcells": round(pg, 1), "ms_per_step_update": round(pms / Tp, 4),
                                           "hbm_gbs_eff": round(pg * 12, 1),
                                           "speedup_tb_vs_plain": round(gcells / pg, 2)}
        pplan.close()
        log("[bench] plain: %.1f GCell/s" % pg)
    plan.close()
    del x, p
    torch.cuda.empty_cache()

    if not args.quick:
        # the same problem in Table 2's physical Hotspot 2D form (its own workload inputs)
        w6 = WORKLOADS["hotspot2d_phys_16384"]
        x6 = torch.from_numpy(w6.field()).to(dev)
        p6 = torch.from_numpy(w6.power()).to(dev)
        pl6 = S.Plan(S.HOTSPOT_PHYS, w6.shape)
        pl6.run(x6, w6.coeffs, 24, p6)
        ms6 = time_call(lambda: pl6.run(x6, w6.coeffs, w6.T, p6), stream, 2)
        g6 = w6.cells * w6.T / (ms6 * 1e-3) / 1e9
        study["hotspot2d_phys_16384"] = model_row(S, pl6, w6.T, ms6, 2, 2, (w6.nx, w6.ny, 1), (256, 0))
        t6 = pl6.tuning
        extras["hotspot2d_phys_16384"] = {"gcells": round(g6, 1), "ms_per_run": round(ms6, 2),
                                          "k": t6["k"], "seg_len": t6["seg_len"],
                                          "pct_single_pass_roofline": round(100 * g6 / (HBM_PEAK_GBS / 12), 1),
                                          # Table 2's 15 FLOP per cell update: 2 adds, 2 FMAs for the
                                          # differences, 1 subtraction, 4 FMAs
                                          "roofline": run_roofline(w6.nx, w6.ny, w6.T, t6["k"],
                                                                   smallest_at_least([4, 8, 12, 16]), t6["seg_len"],
                                                                   1, 2, 15, ms6)}
        pl6.close()
        del x6, p6
        torch.cuda.empty_cache()
        log("[bench] physical hotspot 2D: %.1f GCell/s" % g6)

        # radius-2 star stencil (Eq. 1, Eq. 2 with rad = 2), 2D diffusion form, 16384^2, T = 1000
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
        pp7 = S.StarPlan(w7["rad"], (w7["ny"], w7["nx"]), {"variant": 1})
        msp7 = time_call(lambda: pp7.run(x7, wt7, 20), stream, 1)
        gp7 = c7 * 20 / (msp7 * 1e-3) / 1e9
        study["star2d_r2_16384"] = model_row(S, pl7, w7["T"], ms7, 2, 1, (w7["nx"], w7["ny"], 1), (256, 0),
                                             rad=w7["rad"])
        extras["star2d_r2_16384"] = {"gcells": round(g7, 1), "ms_per_run": round(ms7, 2), "k": t7["k"],
                                     "seg_len": t7["seg_len"], "gcells_one_step": round(gp7, 1),
                                     "pct_single_pass_roofline": round(100 * g7 / (HBM_PEAK_GBS / 8), 1),
                                     # a multiply and 4r FMAs per cell update: 8r + 1 FLOP
                                     "roofline": run_roofline(w7["nx"], w7["ny"], w7["T"], t7["k"],
                                                              smallest_at_least([1, 2, 4, 8]), t7["seg_len"],
                                                              w7["rad"], 1, 8 * w7["rad"] + 1, ms7)}
        pl7.close()
        pp7.close()
        del x7
        torch.cuda.empty_cache()
        log("[bench] radius-2 star 2D: %.1f GCell/s (one step per pass %.1f)" % (g7, gp7))

    if not args.quick:
        # 3D diffusion 512^3, 200 steps: temporal-blocked vs plain
        w3 = WORKLOADS["diffusion3d_512"]
        x3 = torch.from_numpy(w3.field()).to(dev)
        pl3 = S.Plan(DIFFUSION, w3.shape)
        pl3.run(x3, w3.coeffs, 8)
        ms3 = time_call(lambda: pl3.run(x3, w3.coeffs, w3.T), stream, 2)
        g3 = w3.cells * w3.T / (ms3 * 1e-3) / 1e9
        pp3 = S.Plan(DIFFUSION, w3.shape, {"variant": 1})
        msp3 = time_call(lambda: pp3.run(x3, w3.coeffs, 40), stream, 1)
        gp3 = w3.cells * 40 / (msp3 * 1e-3) / 1e9
        study["diffusion3d_512"] = model_row(S, pl3, w3.T, ms3, 3, 1, (w3.nx, w3.ny, w3.nz),
                                             (pl3.tuning["bsize_x"], pl3.tuning["bsize_y"]))
        extras["diffusion3d_512"] = {"gcells_tb": round(g3, 1), "ms_tb": round(ms3, 2), "k": pl3.tuning["k"],
                                     "gcells_plain": round(gp3, 1),
                                     "pct_single_pass_roofline": round(100 * g3 / (HBM_PEAK_GBS / 8), 1)}
        pl3.close(); pp3.close()
        del x3
        log("[bench] 3D: tb %.1f plain %.1f GCell/s" % (g3, gp3))

        # small 2D diffusion 256^2, 16 steps (launch-latency bound)
        w1 = WORKLOADS["diffusion2d_256"]
        x1 = torch.from_numpy(w1.field()).to(dev)
        pl1 = S.Plan(DIFFUSION, w1.shape)
        pl1.run(x1, w1.coeffs, w1.T)
        ms1 = time_call(lambda: pl1.run(x1, w1.coeffs, w1.T), stream, 20)
        study["diffusion2d_256"] = model_row(S, pl1, w1.T, ms1, 2, 1, (w1.nx, w1.ny, 1), (256, 0))
        extras["diffusion2d_256"] = {"us_per_run": round(ms1 * 1e3, 1),
                                     "gcells": round(w1.cells * w1.T / (ms1 * 1e-3) / 1e9, 1)}
        pl1.close()

        # adjoint: hotspot 3D 256^3, 400 steps, checkpoints every 20 steps
        w5 = WORKLOADS["hotspot3d_256_adjoint"]
        x5 = torch.from_numpy(w5.field()).to(dev)
        p5 = torch.from_numpy(w5.power()).to(dev)
        y5 = torch.from_numpy(w5.target()).to(dev)
        pl5 = S.Plan(HOTSPOT, w5.shape)
        xs = x5.clone()
        pl5.run(xs, w5.coeffs, 4, p5)
        xs.copy_(x5)
        fwd_ms = time_call(lambda: pl5.run_ckpt(xs, w5.coeffs, w5.T, w5.ckpt_every, p5), stream, 1)
        study["hotspot3d_256"] = model_row(S, pl5, w5.T, fwd_ms, 3, 2, (w5.nx, w5.ny, w5.nz),
                                             (pl5.tuning["bsize_x"], pl5.tuning["bsize_y"]))
        cot = (xs - y5).contiguous()
        gx = torch.empty_like(x5)
        gp = torch.empty_like(x5)
        adj_ms = time_call(lambda: pl5.adjoint(cot, w5.coeffs, w5.T, gx, gp, p5, 0), stream, 1)
        t0 = time.perf_counter()
        pl5.adjoint(cot, w5.coeffs, w5.T, gx, gp, p5, 1)
        torch.cuda.synchronize()
        adj_rc_ms = (time.perf_counter() - t0) * 1e3
        extras["hotspot3d_256_adjoint"] = {
            "fwd_ckpt_ms": round(fwd_ms, 2), "adjoint_ms": round(adj_ms, 2),
            "adjoint_recompute_ms": round(adj_rc_ms, 2), "ratio_adjoint_fwd": round(adj_ms / fwd_ms, 2),
            "ratio_recompute_fwd": round(adj_rc_ms / fwd_ms, 2),
            "gcells_fwd": round(w5.cells * w5.T / (fwd_ms * 1e-3) / 1e9, 1), "k": pl5.tuning["k"]}
        pl5.close()
        del x5, p5, y5, xs, cot, gx, gp
        log("[bench] adjoint: fwd %.2f ms adj %.2f ms" % (fwd_ms, adj_ms))

        # batched: 64 uneven grids in one persistent launch (graph replay)
        grids = batch_grids()
        xs = [torch.from_numpy(g.field()).to(dev) for g in grids]
        cfs = [SETS[g.coef_set] for g in grids]
        ts = [g.T for g in grids]
        cache = S.run_batched(xs, cfs, ts)
        torch.cuda.synchronize()
        bms = time_call(lambda: S.run_batched(xs, cfs, ts, cache=cache), stream, 2)
        upd = sum(g.cells * g.T for g in grids)
        extras["batched_64"] = {"ms": round(bms, 2), "updates": upd,
                                "gcells_aggregate": round(upd / (bms * 1e-3) / 1e9, 1)}
        S.stencil_batch_destroy(cache)
        del xs
        log("[bench] batched: %.1f GCell/s aggregate" % (upd / (bms * 1e-3) / 1e9))

    out["other_workloads"] = extras
    out["model_accuracy"] = study
    if not args.no_cpu:
        log("[bench] CPU oracle baseline")
        out["cpu_baseline"] = cpu_baseline(wl)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
