// runtime.cpp -- plan, pass scheduler, cost model, auto-tuner and the C ABI of stencil.h.
//
// Pass scheduling (paper Section 3.2, Eq. 8): T steps run as ceil(T/k) passes; each pass reads
// one buffer and writes the other (Section 2.1 ping-pong).  A pass with fewer than k steps
// runs the same kernel with its surplus levels forwarding their input.  The buffer roles are
// arranged so that the last pass writes the caller's buffer; when the pass count is odd the
// input is first copied to the plan scratch.
#include "runtime.hpp"

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <tuple>

namespace stn {

static thread_local std::string g_last_error;

void set_error(const std::string& msg) { g_last_error = msg; }
stencil_status_t fail(stencil_status_t st, const std::string& msg) {
  set_error(msg);
  return st;
}
stencil_status_t hip_fail(hipError_t e, const char* what) {
  set_error(std::string(what) + ": " + hipGetErrorString(e));
  return e == hipErrorOutOfMemory ? STENCIL_ERR_OUT_OF_MEMORY : STENCIL_ERR_HIP;
}
bool env_flag(const char* name) {
  const char* v = std::getenv(name);
  return v && *v && std::strcmp(v, "0") != 0;
}
bool log_enabled() { return env_flag("STENCIL_LOG"); }

const DeviceInfo& device_info() {
  static DeviceInfo info;
  static std::once_flag once;
  std::call_once(once, [] {
    int dev = 0;
    hipDeviceProp_t p;
    if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&p, dev) == hipSuccess) {
      if (p.multiProcessorCount > 0) info.cus = p.multiProcessorCount;
      const double clk = p.clockRate > 0 ? p.clockRate * 1e3 : 2.4e9;
      info.valu_lane_ops = (double)info.cus * 4 * 16 * clk;
    }
  });
  return info;
}

static int round_up(int v, int m) { return (v + m - 1) / m * m; }
static int floor_to(int v, int m) { return v / m * m; }
static int ceil_div(long a, long b) { return (int)((a + b - 1) / b); }

Geom2D geom2d(int K, int nx, int ny, int seg) {
  Geom2D g;
  g.K = K;
  const int W = 64 * kTb2dV;
  g.kr = round_up(K, 4);
  g.cs = floor_to(W - K - g.kr, 4);
  g.ntx = ceil_div(nx, g.cs);
  g.seg = std::max(1, std::min(seg, ny));
  g.nseg = ceil_div(ny, g.seg);
  return g;
}

Geom2D geom_star(int R, int K, int nx, int ny, int seg) {
  Geom2D g;
  g.K = K;
  const int W = 64 * kTb2dV;
  g.kr = round_up(R * K, 4);
  g.cs = floor_to(W - R * K - g.kr, 4);
  g.ntx = ceil_div(nx, g.cs);
  g.seg = std::max(1, std::min(seg, ny));
  g.nseg = ceil_div(ny, g.seg);
  return g;
}

Geom3D geom_star3(int R, int K, int nx, int ny, int nz, int segz) {
  Geom3D g;
  g.K = K;
  g.krx = g.kry = R * K;
  g.csx = g.csy = kStar3W - 2 * R * K;
  g.ntx = ceil_div(nx, g.csx);
  g.nty = ceil_div(ny, g.csy);
  g.segz = std::max(1, std::min(segz, nz));
  g.nsegz = ceil_div(nz, g.segz);
  return g;
}

Geom3D geom3d(int K, bool adj, int nx, int ny, int nz, int segz) {
  Geom3D g;
  g.K = K;
  const int WX = 64 * kTb3dV;
  const int WY = adj ? kTb3dAdjWY : kTb3dWY;
  g.krx = round_up(K, 2);
  g.csx = floor_to(WX - K - g.krx, 2);
  g.kry = K;
  g.csy = WY - 2 * K;
  // Grids at least one window wide (high) place the first and last window of the axis flush
  // with the grid edge, where the clamp costs next to nothing; the tiles between are ordinary
  // overlapped tiles.  x also needs an even width, so every window starts on an 8-byte
  // boundary.
  g.ax = (nx >= WX && (nx % 2) == 0) ? 1 : 0;
  // an even grid narrower than a window: one window flush with x = 0 (ax = 2)
  if (nx < WX && (nx % 2) == 0) g.ax = 2;
  g.ay = (ny >= WY) ? 1 : 0;
  if (g.ax == 2) {
    g.fx = 0;
    g.ntx = 1;
  } else if (g.ax) {
    g.fx = floor_to(WX - K, 2);
    g.ntx = nx == WX ? 1 : (nx <= 2 * g.fx ? 2 : 2 + ceil_div(nx - 2 * g.fx, g.csx));
  } else {
    g.ntx = ceil_div(nx, g.csx);
  }
  if (g.ay) {
    g.fy = WY - K;
    g.nty = ny == WY ? 1 : (ny <= 2 * g.fy ? 2 : 2 + ceil_div(ny - 2 * g.fy, g.csy));
  } else {
    g.nty = ceil_div(ny, g.csy);
  }
  g.segz = std::max(1, std::min(segz, nz));
  g.nsegz = ceil_div(nz, g.segz);
  return g;
}

// The paper's model (Eq. 6-8) counts external-memory cells including the overlapped halos;
// on the GPU a pass also costs VALU time for the redundantly computed halo cells, so a pass is
// priced as max(memory, arithmetic) after wave quantisation, plus a launch overhead.
double model_time_2d(const Geom2D& g, int nx, int ny, long T, bool hot, bool adj, bool phys, ModelParts* parts) {
  const DeviceInfo& d = device_info();
  const int W = 64 * kTb2dV;
  const long passes = (T + g.K - 1) / g.K;
  const double tiles = (double)g.ntx * g.nseg;
  const double rows = (double)g.seg + 2.0 * g.K;  // streamed rows per tile
  const int nread = (hot && !adj) ? 2 : 1;
  const double bytes = tiles * rows * W * 4.0 * nread + (double)nx * ny * 4.0 * (adj && hot ? 3 : 1);
  // VALU instructions per cell and level (the physical hotspot formula takes 9 rounded
  // operations where the weighted sum takes 5)
  const double ops_per_cell = phys ? 9.5 : (adj ? 5.5 : 5.5) + (hot && !adj ? 1.25 : 0.0);
  const double ops = tiles * rows * W * g.K * ops_per_cell;
  const double slots = (double)d.cus * 4 * 2;  // two 64-lane waves per SIMD
  const double rounds = std::ceil(tiles / slots);
  const double quant = tiles / (rounds * slots);
  // Latency hiding: with fewer tiles than about two per wave slot, each SIMD holds too few
  // waves for its whole life (measured: 1917 tiles run at ~0.75 of the rate of 6106); floored
  // at 0.5, below which the pipeline latency below bounds the pass instead.
  const double conc = std::max(0.5, std::min(1.0, std::sqrt(tiles / (2.0 * slots))));
  const double tm = bytes / (d.hbm_gbs * 1e9 * d.achievable_frac);
  // (wave quantisation applies from the second round on: a single partial round is bounded by
  // the pipeline latency below, not by the idle slots)
  const double ta = ops / (d.valu_lane_ops * 0.8) / ((rounds > 1 ? quant : 1.0) * conc);
  // Pipeline latency: one wave streams its tile's rows in order, each row step a chain of K
  // dependent level updates, so a pass takes at least rows x (0.06 + 0.095 K) us however few
  // tiles there are (fitted on a 256^2 grid, where a pass of K = 4 over 16 rows takes 7.8 us,
  // and of K = 8 over 24 rows 16 us, launch included).
  const double tl = rows * (0.06e-6 + 0.095e-6 * g.K);
  if (parts) *parts = ModelParts{passes * tm, passes * std::max(ta, tl)};
  return passes * (std::max(std::max(tm, ta), tl) + 1e-6);
}

// Radius-R star passes: the same pricing with a halo of R*K rows and columns per side, and
// 4R+1 FMAs plus R DPP moves per side (per 4 cells) for each computed cell and level.
double model_time_star(const Geom2D& g, int R, int nx, int ny, long T, ModelParts* parts) {
  const DeviceInfo& d = device_info();
  const int W = 64 * kTb2dV;
  const long passes = (T + g.K - 1) / g.K;
  const double tiles = (double)g.ntx * g.nseg;
  const double bytes = tiles * (g.seg + 2.0 * R * g.K) * W * 4.0 + (double)nx * ny * 4.0;
  const double ops = tiles * W * (g.seg + (double)R * g.K) * g.K * (4.0 * R + 1.0 + 0.5 * R);
  const double slots = (double)d.cus * 4 * 2;
  const double rounds = std::ceil(tiles / slots);
  const double quant = tiles / (rounds * slots);
  const double tm = bytes / (d.hbm_gbs * 1e9 * d.achievable_frac);
  const double ta = ops / (d.valu_lane_ops * 0.8) / quant;
  if (parts) *parts = ModelParts{passes * tm, passes * ta};
  return passes * (std::max(tm, ta) + 4e-6);
}

// Radius-R 3D star passes: every workgroup reads its 64 x 64 window over segz + 2RK planes and
// computes 6R+1 FMAs per window cell and level over segz + K(2R+1) pipeline iterations; one
// workgroup per CU.
double model_time_star3(const Geom3D& g, int R, int nx, int ny, int nz, long T, ModelParts* parts) {
  const DeviceInfo& d = device_info();
  const double W2 = (double)kStar3W * kStar3W;
  const long passes = (T + g.K - 1) / g.K;
  const double tiles = (double)g.ntx * g.nty * g.nsegz;
  const double bytes = tiles * (g.segz + 2.0 * R * g.K) * W2 * 4.0 + (double)nx * ny * nz * 4.0;
  const double iters = g.segz + (double)g.K * (2 * R + 1);
  const double ops = tiles * W2 * iters * g.K * (6.0 * R + 1.0 + 2.0 * R);
  const double rounds = std::ceil(tiles / d.cus);
  const double quant = tiles / (rounds * d.cus);
  const double tm = bytes / (d.hbm_gbs * 1e9 * d.achievable_frac);
  const double ta = ops / (d.valu_lane_ops * 0.6) / quant;
  if (parts) *parts = ModelParts{passes * tm, passes * ta};
  return passes * (std::max(tm, ta) + 4e-6);
}

double model_time_3d(const Geom3D& g, int nx, int ny, int nz, long T, bool hot, bool adj, ModelParts* parts) {
  const DeviceInfo& d = device_info();
  const int WX = 64 * kTb3dV;
  const int WY = adj ? kTb3dAdjWY : kTb3dWY;
  const long passes = (T + g.K - 1) / g.K;
  const double tiles = (double)g.ntx * g.nty * g.nsegz;
  const double planes = (double)g.segz + 2.0 * g.K;
  const int nread = (hot && !adj) ? 2 : 1;
  const double bytes = tiles * planes * WX * WY * 4.0 * nread + (double)nx * ny * nz * 4.0 * (adj && hot ? 3 : 1);
  const double ops = tiles * planes * WX * WY * g.K * (7.5 + (hot && !adj ? 2.0 : 0.0));
  const double slots = (double)d.cus * 1;  // one 512-thread workgroup per CU at these register counts
  const double rounds = std::ceil(tiles / slots);
  const double quant = tiles / (rounds * slots);
  const double tm = bytes / (d.hbm_gbs * 1e9 * d.achievable_frac);
  const double ta = ops / (d.valu_lane_ops * 0.6) / quant;
  if (parts) *parts = ModelParts{passes * tm, passes * ta};
  return passes * (std::max(tm, ta) + 4e-6);
}

double model_time_3d_bal(const Geom3D& g, int nx, int ny, int nz, long T, bool hot, bool adj, int nwork,
                         ModelParts* parts) {
  const DeviceInfo& d = device_info();
  const int WX = 64 * kTb3dV;
  const int WY = adj ? kTb3dAdjWY : kTb3dWY;
  const long passes = (T + g.K - 1) / g.K;
  const double units = (double)g.ntx * g.nty * nz;
  const double share = units / nwork;
  // a share is one column segment, or two when it crosses a column boundary
  const double segs = 1.0 + std::min(1.0, share / nz);
  const double planes = nwork * (share + segs * 2.0 * g.K);
  const int nread = (hot && !adj) ? 2 : 1;
  const double bytes = planes * WX * WY * 4.0 * nread + (double)nx * ny * nz * 4.0 * (adj && hot ? 3 : 1);
  const double ops = planes * WX * WY * g.K * (7.5 + (hot && !adj ? 2.0 : 0.0));
  const double rounds = std::ceil((double)nwork / d.cus);
  const double quant = (double)nwork / (rounds * d.cus);
  const double tm = bytes / (d.hbm_gbs * 1e9 * d.achievable_frac);
  const double ta = ops / (d.valu_lane_ops * 0.6) / quant;
  if (parts) *parts = ModelParts{passes * tm, passes * ta};
  return passes * (std::max(tm, ta) + 4e-6);
}

int balanced_nwork3d(int K, bool adj, int nx, int ny, int nz, int mult) {
  const DeviceInfo& d = device_info();
  const Geom3D g = geom3d(K, adj, nx, ny, nz, nz);
  const long units = (long)g.ntx * g.nty * nz;
  const long most = std::max(1L, units / (4L * K + 4));  // shares of at least ~4 pipeline depths
  return (int)std::max(1L, std::min((long)d.cus * mult, most));
}

int pick_seg2d(int K, int nx, int ny, int waves_per_cu) {
  const DeviceInfo& d = device_info();
  const Geom2D g0 = geom2d(K, nx, ny, ny);
  const long slots = (long)d.cus * waves_per_cu;
  // smallest number of y-tiles that fills the device at least once, rounded so the last round
  // of waves is as full as possible; never segments shorter than 2K rows, except on grids so
  // small that even 2-row segments fit one round of waves: those passes are bound by the
  // pipeline latency of a tile's seg + 2K rows, so shorter segments win there (256^2, k = 4,
  // 16 steps: 22.3 us at 2-row segments, 23.6 at 4, 30.9 at 8)
  const bool tiny = (double)g0.ntx * ceil_div(ny, 2) <= (double)slots;
  const int min_seg = tiny ? 2 : 2 * K;
  int best_seg = ny;
  double best = 1e300;
  for (int nseg = 1; nseg <= std::max(1, ny / std::max(1, min_seg)); ++nseg) {
    const int seg = ceil_div(ny, nseg);
    const int real = ceil_div(ny, seg);
    const double tiles = (double)g0.ntx * real;
    const double rounds = std::ceil(tiles / slots);
    const double per_tile = seg + 2.0 * K + 2.0;  // streamed rows incl. pipeline fill
    const double cost = rounds * per_tile;        // time ~ rounds x rows per wave
    if (cost < best * 0.999) {
      best = cost;
      best_seg = seg;
    }
    if (tiles > 64.0 * slots) break;
  }
  return best_seg;
}

int pick_segz3d(int K, bool adj, int nx, int ny, int nz, int wgs_per_cu) {
  const DeviceInfo& d = device_info();
  const Geom3D g0 = geom3d(K, adj, nx, ny, nz, nz);
  const long slots = (long)d.cus * wgs_per_cu;
  int best = nz;
  double bestc = 1e300;
  for (int ns = 1; ns <= std::max(1, nz / std::max(1, 2 * K)); ++ns) {
    const int segz = ceil_div(nz, ns);
    const int real = ceil_div(nz, segz);
    const double tiles = (double)g0.ntx * g0.nty * real;
    const double rounds = std::ceil(tiles / slots);
    const double cost = rounds * (segz + 2.0 * K + 2.0);
    if (cost < bestc * 0.999) {
      bestc = cost;
      best = segz;
    }
    if (tiles > 64.0 * slots) break;
  }
  return best;
}

DevCoef dev_coef(const stencil_coeffs_t& c, bool adjoint, bool phys) {
  DevCoef d;
  if (phys) {
    // Table 2's physical Hotspot 2D parameters (see DevCoef): sdc in cp, Rx_1 in ce, Ry_1 in
    // cs, Rz_1 in c_amb, TEMP_AMB in t_amb
    d.c0 = 0.0f;
    d.wx_m = d.wx_p = c.ce;
    d.wy_m = d.wy_p = c.cs;
    d.wz_m = c.c_amb;
    d.wz_p = 0.0f;
    d.cp = c.cp;
    d.kamb = c.t_amb;
    return d;
  }
  d.c0 = c.cc;
  if (!adjoint) {
    d.wx_m = c.cw; d.wx_p = c.ce; d.wy_m = c.cn; d.wy_p = c.cs; d.wz_m = c.cb; d.wz_p = c.ca;
  } else {
    d.wx_m = c.ce; d.wx_p = c.cw; d.wy_m = c.cs; d.wy_p = c.cn; d.wz_m = c.ca; d.wz_p = c.cb;
  }
  d.cp = c.cp;
  d.kamb = c.c_amb * c.t_amb;  // rounded once in FP32
  return d;
}

bool coeffs_finite(const stencil_coeffs_t& c) {
  const float v[] = {c.cc, c.cw, c.ce, c.cn, c.cs, c.cb, c.ca, c.cp, c.c_amb, c.t_amb};
  for (float x : v)
    if (!std::isfinite(x)) return false;
  return true;
}

}  // namespace stn

using namespace stn;

namespace {

bool aligned16(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 15) == 0; }

// Fault injection for tests of the error paths: STENCIL_FAULT_INJECT=<pass index> makes the
// pass scheduler report a HIP error before launching that pass (no device work is skipped
// silently: the call returns STENCIL_ERR_HIP).
int fault_pass() {
  const char* v = std::getenv("STENCIL_FAULT_INJECT");
  return v && *v ? std::atoi(v) : -1;
}

// Debug aid for tests: STENCIL_DEBUG_POISON=1 fills the plan's ping-pong scratch with NaN
// before every run, so a read of scratch cells that no pass has written turns the result NaN.
hipError_t poison_scratch(const stencil_plan_s* p) {
  if (!env_flag("STENCIL_DEBUG_POISON")) return hipSuccess;
  return launch_fill(p->scratch, p->cells, __builtin_nanf(""), p->stream);
}

KMode form_mode(stencil_form_t f) {
  return f == STENCIL_HOTSPOT ? KM_HOT : (f == STENCIL_HOTSPOT_PHYS ? KM_PHYS : KM_DIFF);
}
KMode fwd_mode(const stencil_plan_s* p) { return form_mode(p->form); }

int star_inst(int ndim, int R, const int** ks) {
  return ndim == 3 ? star3_instantiated(R, ks) : star_instantiated(R, ks);
}

// Smallest instantiated K >= k of the radius-R star kernels (the largest if none is).
int star_k_for(int ndim, int R, int k) {
  const int* ks;
  const int n = star_inst(ndim, R, &ks);
  for (int i = 0; i < n; ++i)
    if (ks[i] >= k) return ks[i];
  return ks[n - 1];
}

// Smallest instantiated K >= k.
int inst_k_for(int ndim, KMode m, int k) {
  const int* ks;
  const int n = tb_instantiated(ndim, m, &ks);
  for (int i = 0; i < n; ++i)
    if (ks[i] >= k) return ks[i];
  return ks[n - 1];
}

// Interior rectangle of a 2D pass: tiles whose window lies inside the grid in x and whose
// rows (with the keff-row halo) stay clear of the first and last grid row, i.e. the tiles for
// which the kernel takes its edge-free body.  Both conditions are per axis, so those tiles form
// a rectangle [*x0, *x1) x [*y0, *y1) of tile indices (empty if x0 >= x1 or y0 >= y1).
// Segments cover the output rows [ylo, yhi).
void interior_rect2d(const Geom2D& g, int nx, int ny, int keff, int ylo, int yhi, int* x0, int* x1, int* y0,
                     int* y1) {
  const int W = 64 * kTb2dV;
  *x0 = g.ntx; *x1 = 0; *y0 = g.nseg; *y1 = 0;
  for (int tx = 0; tx < g.ntx; ++tx) {
    const int ws = tx * g.cs - g.kr;
    if (ws >= 0 && ws + W <= nx) { *x0 = std::min(*x0, tx); *x1 = std::max(*x1, tx + 1); }
  }
  for (int sg = 0; sg < g.nseg; ++sg) {
    const int r0 = ylo + sg * g.seg, r1 = std::min(r0 + g.seg, yhi);
    if (r0 - keff > 0 && r1 + keff < ny) { *y0 = std::min(*y0, sg); *y1 = std::max(*y1, sg + 1); }
  }
}

// One pass of keff fused steps from src to dst.
hipError_t run_star_pass(const stencil_plan_s* p, int K, int keff, const float* src, float* dst) {
  if (p->ndim == 3) {
    const Geom3D g = geom_star3(p->rad, K, p->nx, p->ny, p->nz, p->tuning.seg_len);
    Star3dArgs a;
    a.src = src; a.dst = dst;
    a.nx = p->nx; a.ny = p->ny; a.nz = p->nz; a.keff = keff;
    a.cs = g.csx; a.ntx = g.ntx; a.nty = g.nty; a.segz = g.segz; a.nsegz = g.nsegz;
    a.power = p->star_power;
    a.cf = p->star3_cf;
    return launch_star3d(p->rad, K, a, p->stream);
  }
  const Geom2D g = geom_star(p->rad, K, p->nx, p->ny, p->tuning.seg_len);
  Star2dArgs a;
  a.src = src; a.dst = dst;
  a.nx = p->nx; a.ny = p->ny; a.keff = keff;
  a.cs = g.cs; a.kr = g.kr; a.ntx = g.ntx; a.seg = g.seg; a.nseg = g.nseg;
  a.aligned = ((p->nx & 3) == 0) && aligned16(src) && aligned16(dst) &&
                      (!p->star_power || aligned16(p->star_power)) ? 1 : 0;
  a.power = p->star_power;
  a.cf = p->star_cf;
  return launch_star2d(p->rad, K, a, p->stream);
}

// Nontemporal output stores in the 2D temporal-blocked and the one-step kernels for fields
// above 128 MiB, half the 256 MB last-level cache, with rows shorter than 2^29 cells (the byte
// range of the buffer store that carries the hint).  Measured against plain stores on one
// device: +1.1% (hotspot 16384^2, k = 12), +1.7% and +4.2% (one-step 16384^2 and 512^3); with
// the hint on every grid, 256^3 (64 MiB) ran 5-13% slower, since its next pass reads the input
// back from that cache.  The 3D temporal-blocked kernel keeps plain stores: with the hint it
// gained 0.6% at its tuned k = 4 on 512^3 and lost 3-5% at k = 5 and 6.
constexpr size_t kStreamStoreBytes = size_t(128) << 20;
int stream_stores(const stencil_plan_s* p) {
  return p->cells * sizeof(float) > kStreamStoreBytes && p->nx < (1 << 29) ? 1 : 0;
}

// One pass of keff fused steps from src to dst.  Output cells along the streamed axis (y in
// 2D, z in 3D) are [lo, hi); hi < 0 means every cell (a slab pass narrows it to its interior).
hipError_t run_pass(const stencil_plan_s* p, KMode m, int K, int keff, const float* src, float* dst,
                    const float* power, float* gp, const DevCoef& cf, int lo = 0, int hi = -1) {
  if (m == KM_STAR) return run_star_pass(p, K, keff, src, dst);
  const bool full = (keff == K);
  if (p->ndim == 2) {
    if (hi < 0) hi = p->ny;
    const Geom2D g = geom2d(K, p->nx, hi - lo, p->tuning.seg_len);
    Tb2dArgs a;
    a.src = src; a.dst = dst; a.power = power; a.gp = gp;
    a.nx = p->nx; a.ny = p->ny; a.keff = keff;
    a.cs = g.cs; a.kr = g.kr; a.ntx = g.ntx; a.seg = g.seg; a.nseg = g.nseg;
    a.aligned = ((p->nx & 3) == 0) && aligned16(src) && aligned16(dst) && (!power || aligned16(power)) &&
                (!gp || aligned16(gp)) ? 1 : 0;
    a.stream = stream_stores(p);
    a.cf = cf;
    a.part = 0;
    a.ylo = lo;
    a.yhi = hi;
    interior_rect2d(g, p->nx, p->ny, keff, lo, hi, &a.ix0, &a.ix1, &a.iy0, &a.iy1);
    const long interior = (a.ix1 > a.ix0 && a.iy1 > a.iy0) ? (long)(a.ix1 - a.ix0) * (a.iy1 - a.iy0) : 0;
    const long total = (long)g.ntx * g.nseg;
    // Split when the interior kernel has enough tiles to fill the device and some tiles are
    // edge tiles: the interior kernel, free of edge code, needs fewer registers; the frame
    // kernel runs beside it on the side stream (fork/join through events).
    if (!a.aligned || !p->side || interior < 1024 || interior == total) {
      a.ix0 = a.ix1 = a.iy0 = a.iy1 = 0;
      return launch_tb2d(K, m, full, a, p->stream);
    }
    hipError_t e = hipEventRecord(p->ev_fork, p->stream);
    if (e == hipSuccess) e = hipStreamWaitEvent(p->side, p->ev_fork, 0);
    if (e != hipSuccess) return e;
    Tb2dArgs fr = a;
    fr.part = 2;
    e = launch_tb2d(K, m, full, fr, p->side);
    if (e == hipSuccess) e = hipEventRecord(p->ev_join, p->side);
    if (e != hipSuccess) return e;
    a.part = 1;
    e = launch_tb2d(K, m, full, a, p->stream);
    if (e != hipSuccess) return e;
    return hipStreamWaitEvent(p->stream, p->ev_join, 0);
  }
  const bool adj = (m == KM_ADJ || m == KM_ADJ_ACC);
  if (hi < 0) hi = p->nz;
  Geom3D g = geom3d(K, adj, p->nx, p->ny, p->nz, p->tuning.seg_len);
  g.segz = std::max(1, std::min(g.segz, hi - lo));
  g.nsegz = ceil_div(hi - lo, g.segz);
  Tb3dArgs a;
  a.src = src; a.dst = dst; a.power = power; a.gp = gp;
  a.nx = p->nx; a.ny = p->ny; a.nz = p->nz; a.keff = keff;
  a.csx = g.csx; a.csy = g.csy; a.krx = g.krx; a.kry = g.kry; a.ntx = g.ntx; a.nty = g.nty;
  a.segz = g.segz; a.nsegz = g.nsegz;
  a.ax = g.ax; a.ay = g.ay; a.fx = g.fx; a.fy = g.fy;
  a.nwork = p->nwork3d;
  // 8-byte vector accesses of the field, the power map (hotspot) and grad_p (adjoint)
  const uintptr_t bits = reinterpret_cast<uintptr_t>(src) | reinterpret_cast<uintptr_t>(dst) |
                         reinterpret_cast<uintptr_t>(power) | reinterpret_cast<uintptr_t>(gp);
  a.aligned = ((p->nx & 1) == 0) && (bits & 7) == 0 ? 1 : 0;
  a.zlo = lo;
  a.zhi = hi;
  a.cf = cf;
  return launch_tb3d(K, m, full, a, p->stream);
}

// Planes per strip of the one-step 3D kernel (one one-wave workgroup per 256-column chunk, row
// and strip): the longest of 16, 32, ..., 256 planes that divides nz evenly and still gives at
// least 16 workgroups per CU, else 32.  Measured (diffusion, TB/s, at the chosen length against
// 32 planes): 512^3 4.30 (128) / 4.02, 1024 x 512^2 4.44 (256) / 4.12, 384^3 3.23 (64) / 3.11,
// 256^3 5.26 (16) / 3.98 (that grid stays in the last-level cache), 256 x 1024^2 4.03 (256) /
// 4.01; unequal strips cost (160 x 600 x 700: 3.00 at 64 planes, 3.47 at 32), and 640^3 runs at
// 3.80 (128) against 3.91.
int plain_strip3d(int chunks, int ny, int nz) {
  const long cols = (long)chunks * ny;
  const long want = 16L * device_info().cus;
  int best = 0;
  for (int mr = 16; mr <= 256; mr *= 2)
    if (nz % mr == 0 && cols * (nz / mr) >= want) best = mr;
  return best ? best : 32;
}

hipError_t run_plain_step(const stencil_plan_s* p, KMode m, const float* src, float* dst, const float* power,
                          float* gp, const DevCoef& cf) {
  PlainArgs a;
  a.src = src; a.dst = dst; a.power = power; a.gp = gp;
  a.nx = p->nx; a.ny = p->ny; a.nz = p->nz; a.ndim = p->ndim;
  a.chunks = (p->nx + 255) / 256;
  a.vec = ((p->nx & 3) == 0) && aligned16(src) && aligned16(dst) && (!power || aligned16(power)) &&
          (!gp || aligned16(gp)) ? 1 : 0;
  a.stream = stream_stores(p);
  a.mr3 = p->ndim == 3 ? plain_strip3d(a.chunks, p->ny, p->nz) : 1;
  a.cf = cf;
  return launch_plain(m, a, p->stream);
}

// Split T steps into passes of at most kmax steps (the first passes full).
std::vector<int> split_steps(int T, int kmax) {
  std::vector<int> v;
  for (int done = 0; done < T; done += kmax) v.push_back(std::min(kmax, T - done));
  return v;
}

// Run the pass sequence `steps` starting from `first_src` (holding x_0), ending in `out`.
// `alt` is the second ping-pong buffer.  If first_src == out and the pass count is odd, the
// input is copied to alt first.  gp (adjoint accumulation) is passed to every pass.
stencil_status_t run_sequence(stencil_plan_s* p, KMode m, bool plain, int K, const std::vector<int>& steps,
                              const float* first_src, float* out, float* alt, const float* power, float* gp,
                              const DevCoef& cf, int* pass_counter) {
  const size_t bytes = p->cells * sizeof(float);
  const int P = (int)steps.size();
  if (P == 0) {
    if (first_src != out) {
      hipError_t e = hipMemcpyAsync(out, first_src, bytes, hipMemcpyDeviceToDevice, p->stream);
      if (e != hipSuccess) return hip_fail(e, "hipMemcpyAsync");
    }
    return STENCIL_OK;
  }
  const float* src = first_src;
  // Pass i writes `out` when (P - 1 - i) is even.
  if (first_src == out && (P % 2) == 1) {
    hipError_t e = hipMemcpyAsync(alt, out, bytes, hipMemcpyDeviceToDevice, p->stream);
    if (e != hipSuccess) return hip_fail(e, "hipMemcpyAsync");
    src = alt;
  }
  const int fi = fault_pass();
  for (int i = 0; i < P; ++i) {
    float* dst = ((P - 1 - i) % 2 == 0) ? out : alt;
    if (dst == src) return fail(STENCIL_ERR_INTERNAL, "pass scheduler produced an in-place pass");
    if (fi >= 0 && *pass_counter == fi) {
      ++*pass_counter;
      return fail(STENCIL_ERR_HIP, "injected fault (STENCIL_FAULT_INJECT) at pass " + std::to_string(fi));
    }
    ++*pass_counter;
    hipError_t e;
    if (plain) {
      e = run_plain_step(p, m, src, dst, power, gp, cf);  // plain passes are single steps
    } else {
      // a pass that fuses fewer steps than K runs on the smallest instantiation that holds
      // them: surplus levels would only forward their input at the full pass's cost
      const int Ki = steps[i] < K ? (m == KM_STAR ? star_k_for(p->ndim, p->rad, steps[i]) : inst_k_for(p->ndim, m, steps[i]))
                                  : K;
      e = run_pass(p, m, Ki, steps[i], src, dst, power, gp, cf);
    }
    if (e != hipSuccess) return hip_fail(e, "kernel launch");
    src = dst;
  }
  return STENCIL_OK;
}

// Kernel/K selection for a forward or adjoint run of the plan.
void resolve_k(const stencil_plan_s* p, KMode m, int* K, bool* plain) {
  *plain = (p->tuning.variant == 1);
  int k = p->tuning.k > 0 ? p->tuning.k : 1;
  const int kmax = tb_max_k(p->ndim, m);
  if (k > kmax) k = kmax;
  *K = inst_k_for(p->ndim, m, k);
}

struct TuneKey {
  int form, ndim, nx, ny, nz;
  bool operator<(const TuneKey& o) const {
    return std::tie(form, ndim, nx, ny, nz) < std::tie(o.form, o.ndim, o.nx, o.ny, o.nz);
  }
};
std::mutex g_tune_mu;
struct TuneResult {
  stencil_tuning_t t;
  int nwork;
  int adj_k, adj_seg, adj_nwork;  // the transposed pass's own blocking
};
std::map<TuneKey, TuneResult> g_tune_cache;

// Tuning results persist across processes when STENCIL_TUNE_CACHE names a file: it is read
// once, before the first tuning, and every new result is appended to it, one line per shape
// ("form ndim nx ny nz : variant k vec bsize_x bsize_y seg_len nwork adj_k adj_seg adj_nwork").
// A profiler run can then reuse exactly the blockings a timed run chose.
const char* tune_cache_path() {
  const char* v = std::getenv("STENCIL_TUNE_CACHE");
  return (v && *v) ? v : nullptr;
}
void load_tune_cache_file() {
  static bool loaded = false;
  if (loaded) return;
  loaded = true;
  const char* path = tune_cache_path();
  if (!path) return;
  FILE* f = std::fopen(path, "r");
  if (!f) return;
  int form, ndim, nx, ny, nz;
  TuneResult r{};
  while (std::fscanf(f, "%d %d %d %d %d : %d %d %d %d %d %d %d %d %d %d", &form, &ndim, &nx, &ny, &nz, &r.t.variant,
                     &r.t.k, &r.t.vec, &r.t.bsize_x, &r.t.bsize_y, &r.t.seg_len, &r.nwork, &r.adj_k, &r.adj_seg,
                     &r.adj_nwork) == 15) {
    r.t.nwork = r.nwork;
    g_tune_cache[TuneKey{form, ndim, nx, ny, nz}] = r;
  }
  std::fclose(f);
}
void save_tune_result(const TuneKey& k, const TuneResult& r) {
  const char* path = tune_cache_path();
  if (!path) return;
  FILE* f = std::fopen(path, "a");
  if (!f) return;
  std::fprintf(f, "%d %d %d %d %d : %d %d %d %d %d %d %d %d %d %d\n", k.form, k.ndim, k.nx, k.ny, k.nz, r.t.variant,
               r.t.k, r.t.vec, r.t.bsize_x, r.t.bsize_y, r.t.seg_len, r.nwork, r.adj_k, r.adj_seg, r.adj_nwork);
  std::fclose(f);
}

// Model-ranked candidates, the best few timed on scratch memory.
stencil_status_t autotune(stencil_plan_s* p, TuneResult* out) {
  const TuneKey key{p->form, p->ndim, p->nx, p->ny, p->nz};
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    load_tune_cache_file();
    auto it = g_tune_cache.find(key);
    if (it != g_tune_cache.end()) {
      *out = it->second;
      return STENCIL_OK;
    }
  }
  const bool hot = p->form != STENCIL_DIFFUSION;  // reads a power map
  const bool phys = p->form == STENCIL_HOTSPOT_PHYS;
  const KMode m = fwd_mode(p);
  const long Tref = 240;  // a step count divisible by every instantiated k
  struct Cand {
    int K, seg;
    double model;
    int nwork;  // 3D balanced launch (seg unused), 0 = tile launch
  };
  std::vector<Cand> cands;
  const int* ks;
  const int nk = tb_instantiated(p->ndim, m, &ks);
  for (int i = 0; i < nk; ++i) {
    const int K = ks[i];
    if (p->ndim == 2) {
      // segment lengths that keep several waves per SIMD busy; odd multiples of 32 rows avoid
      // every tile starting on the same power-of-two row stride
      for (int seg : {96, 128, 160, 192, 224, 288, 352, 480, 608}) {
        if (seg < 2 * K && seg < p->ny) continue;
        const Geom2D g = geom2d(K, p->nx, p->ny, seg);
        cands.push_back({K, g.seg, model_time_2d(g, p->nx, p->ny, Tref, hot, false, phys), 0});
      }
      for (int wpc : {8, 12}) {
        const int seg = pick_seg2d(K, p->nx, p->ny, wpc);
        const Geom2D g = geom2d(K, p->nx, p->ny, seg);
        cands.push_back({K, seg, model_time_2d(g, p->nx, p->ny, Tref, hot, false, phys), 0});
      }
    } else {
      for (int mult : {1, 2}) {
        const int nw = balanced_nwork3d(K, false, p->nx, p->ny, p->nz, mult);
        const Geom3D g = geom3d(K, false, p->nx, p->ny, p->nz, p->nz);
        const int share = (int)ceil_div((long)g.ntx * g.nty * p->nz, nw);
        cands.push_back({K, share, model_time_3d_bal(g, p->nx, p->ny, p->nz, Tref, hot, false, nw), nw});
      }
      for (int wpc : {1, 2}) {
        const int segz = pick_segz3d(K, false, p->nx, p->ny, p->nz, wpc);
        const Geom3D g = geom3d(K, false, p->nx, p->ny, p->nz, segz);
        cands.push_back({K, segz, model_time_3d(g, p->nx, p->ny, p->nz, Tref, hot, false), 0});
      }
      for (int segz : {32, 48, 64, 96, 128}) {
        if (segz > p->nz) continue;
        const Geom3D g = geom3d(K, false, p->nx, p->ny, p->nz, segz);
        cands.push_back({K, g.segz, model_time_3d(g, p->nx, p->ny, p->nz, Tref, hot, false), 0});
      }
    }
  }
  std::sort(cands.begin(), cands.end(), [](const Cand& a, const Cand& b) { return a.model < b.model; });
  // remove duplicates
  std::vector<Cand> all;
  for (const Cand& c : cands) {
    bool dup = false;
    for (const Cand& u : all) dup |= (u.K == c.K && u.seg == c.seg && u.nwork == c.nwork);
    if (!dup) all.push_back(c);
  }
  // Timed set: the three best-modelled candidates of every K (the model ranks the launch
  // shapes of one K well, K against K less so), in model order.
  std::vector<Cand> uniq;
  for (const Cand& c : all) {
    int same_k = 0;
    for (const Cand& u : uniq) same_k += (u.K == c.K);
    if (same_k < 3) uniq.push_back(c);
  }
  stencil_tuning_t best = p->tuning;
  best.variant = 2;
  best.k = uniq[0].K;
  best.seg_len = uniq[0].seg;
  int best_nwork = uniq[0].nwork;
  // adjoint default (untimed): the instantiated adjoint K with the least modelled time, on
  // the forward's segment length and the tile launch
  const KMode am = hot ? KM_ADJ_ACC : KM_ADJ;
  int adj_k = 1, adj_seg = best.seg_len, adj_nwork = 0;
  {
    const int* aks;
    const int nak = tb_instantiated(p->ndim, am, &aks);
    double bm = 1e300;
    for (int i = 0; i < nak; ++i) {
      const double tm =
          p->ndim == 2 ? model_time_2d(geom2d(aks[i], p->nx, p->ny, best.seg_len), p->nx, p->ny, Tref, hot, true)
                       : model_time_3d(geom3d(aks[i], true, p->nx, p->ny, p->nz, best.seg_len), p->nx, p->ny, p->nz,
                                       Tref, hot, true);
      if (tm < bm) {
        bm = tm;
        adj_k = aks[i];
      }
    }
  }
  const bool timed = !env_flag("STENCIL_MODEL_ONLY") && p->cells >= (size_t)1 << 16;
  if (timed) {
    // Time the top candidates on scratch memory.
    // Hotspot trials read a power map of their own: sharing the source buffer would hide a
    // third of the pass's HBM reads and favour small k.
    float* tmp = nullptr;
    float* pw = nullptr;
    const bool have = hipMalloc(&tmp, p->cells * sizeof(float)) == hipSuccess &&
                      (!hot || hipMalloc(&pw, p->cells * sizeof(float)) == hipSuccess);
    if (have) {
      launch_fill(tmp, p->cells, 0.5f, p->stream);
      launch_fill(p->scratch, p->cells, 0.5f, p->stream);
      if (pw) launch_fill(pw, p->cells, 0.0f, p->stream);
      stencil_coeffs_t c{};
      c.cc = 0.5f; c.cw = c.ce = c.cn = c.cs = 0.125f; c.cb = c.ca = 0.0f;
      const DevCoef cf = dev_coef(c, false, phys);
      hipEvent_t e0, e1;
      hipEventCreate(&e0);
      hipEventCreate(&e1);
      const int ntop = (int)uniq.size();
      // Each candidate runs `reps` back-to-back passes (at least ~12 ms of work at 3.5e12
      // updates/s, so launch gaps and timer resolution stay small), in three rounds over the
      // list after a warm-up that brings the clocks up; the best of the rounds counts.
      auto time_cand = [&](const Cand& cd) -> double {
        stencil_plan_s q = *p;
        q.tuning.k = cd.K;
        q.tuning.seg_len = cd.seg;
        q.nwork3d = cd.nwork;
        const double per_pass = (double)cd.K * (double)p->cells;
        const int reps = std::max(2, std::min(192, (int)std::ceil(4.2e10 / per_pass)));
        run_pass(&q, m, cd.K, cd.K, tmp, p->scratch, pw, nullptr, cf);
        hipEventRecord(e0, p->stream);
        for (int r = 0; r < reps; ++r) {
          const bool even = (r % 2) == 0;
          float* s = even ? p->scratch : tmp;
          float* d = even ? tmp : p->scratch;
          run_pass(&q, m, cd.K, cd.K, s, d, pw, nullptr, cf);
        }
        hipEventRecord(e1, p->stream);
        hipEventSynchronize(e1);
        float ms = 0;
        hipEventElapsedTime(&ms, e0, e1);
        return ms > 0 ? reps * per_pass / (ms * 1e-3) : 0.0;  // cell updates / s
      };
      for (int w = 0; w < 3; ++w) time_cand(uniq[0]);
      std::vector<double> rate(ntop, 0.0);
      for (int round = 0; round < 3; ++round)
        for (int i = 0; i < ntop; ++i) rate[i] = std::max(rate[i], time_cand(uniq[i]));
      // Trials of one candidate still vary by about 0.5% from call to call, so every candidate
      // within 0.5% of the fastest counts as a tie, and the tie goes to the best-modelled one
      // (the list is in model order).
      double best_rate = 0;
      for (int i = 0; i < ntop; ++i) {
        if (log_enabled())
          std::fprintf(stderr, "[stencil] tune K=%d seg=%d nwork=%d model=%.3g ms measured=%.1f GCell/s\n",
                       uniq[i].K, uniq[i].seg, uniq[i].nwork, uniq[i].model * 1e3, rate[i] * 1e-9);
        best_rate = std::max(best_rate, rate[i]);
      }
      for (int i = 0; i < ntop; ++i) {
        if (rate[i] >= 0.995 * best_rate) {
          best.k = uniq[i].K;
          best.seg_len = uniq[i].seg;
          best_nwork = uniq[i].nwork;
          break;
        }
      }
      // 2D: the candidate segments are 32 rows apart, so the winner's neighbours 16 rows either
      // side are timed too, and one of them replaces it when it is faster by more than the
      // trial noise (hotspot 16384^2, k = 12: 176 rows ran 1.4% faster than 192).
      if (p->ndim == 2) {
        const Cand win{best.k, best.seg_len, 0.0, 0};
        std::vector<Cand> nb;
        for (int d : {-16, 16}) {
          const int seg = best.seg_len + d;
          if (seg >= 2 * best.k && seg < p->ny) nb.push_back({best.k, seg, 0.0, 0});
        }
        double wr = 0.0;
        std::vector<double> nr(nb.size(), 0.0);
        for (int round = 0; round < 3 && !nb.empty(); ++round) {
          wr = std::max(wr, time_cand(win));
          for (size_t i = 0; i < nb.size(); ++i) nr[i] = std::max(nr[i], time_cand(nb[i]));
        }
        for (size_t i = 0; i < nb.size(); ++i) {
          if (log_enabled())
            std::fprintf(stderr, "[stencil] tune K=%d seg=%d (neighbour of %d) measured=%.1f GCell/s against %.1f\n",
                         nb[i].K, nb[i].seg, win.seg, nr[i] * 1e-9, wr * 1e-9);
          if (nr[i] > 1.005 * wr) {
            wr = nr[i];
            best.seg_len = nb[i].seg;
          }
        }
      }
      // The transposed pass (it also reads and writes grad_p) is timed on candidates of its
      // own: every instantiated K with a few segment lengths and, in 3D, the balanced launch;
      // one round after a warm-up.  (The physical Hotspot 2D form has no transposed pass.)
      if (!phys) {
        const DevCoef acf = dev_coef(c, true);
        const int* aks;
        const int nak = tb_instantiated(p->ndim, am, &aks);
        struct ACand {
          int K, seg, nwork;
        };
        std::vector<ACand> ac;
        for (int i = 0; i < nak; ++i) {
          if (p->ndim == 2) {
            for (int sg : {best.seg_len, 96, 192, 384})
              if (sg <= p->ny || sg == best.seg_len) ac.push_back({aks[i], sg, 0});
          } else {
            for (int sz : {8, 16, 32, 64})
              if (sz <= p->nz) ac.push_back({aks[i], sz, 0});
            ac.push_back({aks[i], p->nz, balanced_nwork3d(aks[i], true, p->nx, p->ny, p->nz, 1)});
          }
        }
        auto time_adj = [&](const ACand& cd) -> double {
          stencil_plan_s q = *p;
          q.tuning.k = cd.K;
          q.tuning.seg_len = cd.seg;
          q.nwork3d = cd.nwork;
          const double per_pass = (double)cd.K * (double)p->cells;
          const int reps = std::max(2, std::min(64, (int)std::ceil(7e9 / per_pass)));
          run_pass(&q, am, cd.K, cd.K, tmp, p->scratch, nullptr, pw, acf);
          hipEventRecord(e0, p->stream);
          for (int r = 0; r < reps; ++r) {
            const bool even = (r % 2) == 0;
            run_pass(&q, am, cd.K, cd.K, even ? p->scratch : tmp, even ? tmp : p->scratch, nullptr, pw, acf);
          }
          hipEventRecord(e1, p->stream);
          hipEventSynchronize(e1);
          float ms = 0;
          hipEventElapsedTime(&ms, e0, e1);
          return ms > 0 ? reps * per_pass / (ms * 1e-3) : 0.0;
        };
        double best_arate = 0;
        for (const ACand& cd : ac) {
          const double r = time_adj(cd);
          if (log_enabled())
            std::fprintf(stderr, "[stencil] tune adjoint K=%d seg=%d nwork=%d measured=%.1f GCell/s\n", cd.K, cd.seg,
                         cd.nwork, r * 1e-9);
          if (r > best_arate) {
            best_arate = r;
            adj_k = cd.K;
            adj_seg = cd.seg;
            adj_nwork = cd.nwork;
          }
        }
      }
      hipEventDestroy(e0);
      hipEventDestroy(e1);
    }
    hipStreamSynchronize(p->stream);
    if (tmp) hipFree(tmp);
    if (pw) hipFree(pw);
    hipGetLastError();
  }
  if (log_enabled())
    std::fprintf(stderr, "[stencil] plan form=%d ndim=%d %dx%dx%d -> k=%d seg=%d nwork=%d\n", p->form, p->ndim, p->nx,
                 p->ny, p->nz, best.k, best.seg_len, best_nwork);
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune_cache[key] = TuneResult{best, best_nwork, adj_k, adj_seg, adj_nwork};
    save_tune_result(key, g_tune_cache[key]);
  }
  *out = TuneResult{best, best_nwork, adj_k, adj_seg, adj_nwork};
  return STENCIL_OK;
}

stencil_status_t check_plan(stencil_plan_t plan) {
  if (!plan) return fail(STENCIL_ERR_INVALID_ARG, "plan is NULL");
  return STENCIL_OK;
}

// Segment length of a radius-R star pass: the fewest row segments that give about two waves
// per SIMD in full rounds, as pick_seg2d does for the radius-1 kernels.
int pick_seg_star(int R, int K, int nx, int ny) {
  const DeviceInfo& d = device_info();
  const Geom2D g0 = geom_star(R, K, nx, ny, ny);
  const long slots = (long)d.cus * 8;
  int best_seg = ny;
  double best = 1e300;
  for (int nseg = 1; nseg <= std::max(1, ny / std::max(1, 2 * R * K)); ++nseg) {
    const int seg = ceil_div(ny, nseg);
    const double tiles = (double)g0.ntx * ceil_div(ny, seg);
    const double cost = std::ceil(tiles / slots) * (seg + 2.0 * R * K + 2.0);
    if (cost < best * 0.999) {
      best = cost;
      best_seg = seg;
    }
    if (tiles > 64.0 * slots) break;
  }
  return best_seg;
}

// Segment length (planes) of a radius-R 3D star pass: whole rounds of one workgroup per CU,
// each workgroup paying K(2R+1) pipeline-fill iterations on top of its planes.
int pick_segz_star3(int R, int K, int nx, int ny, int nz) {
  const DeviceInfo& d = device_info();
  const Geom3D g0 = geom_star3(R, K, nx, ny, nz, nz);
  const double tiles_xy = (double)g0.ntx * g0.nty;
  int best_seg = nz;
  double best = 1e300;
  for (int nseg = 1; nseg <= nz; ++nseg) {
    const int seg = ceil_div(nz, nseg);
    const double wg = tiles_xy * ceil_div(nz, seg);
    const double cost = std::ceil(wg / d.cus) * (seg + (double)K * (2 * R + 1) + 2.0 * R * K);
    if (cost < best * 0.999) {
      best = cost;
      best_seg = seg;
    }
    if (wg > 32.0 * d.cus) break;
  }
  return best_seg;
}

int pick_seg_star_nd(const stencil_plan_s* p, int K) {
  return p->ndim == 3 ? pick_segz_star3(p->rad, K, p->nx, p->ny, p->nz) : pick_seg_star(p->rad, K, p->nx, p->ny);
}

// Blocking of a radius-R star plan: every instantiated K, each on its own segment length, is
// timed on scratch memory (three rounds of at least ~12 ms after a warm-up) and the fastest
// kept; grids below 2^16 cells take K = 4 untimed.
void star_tune(stencil_plan_s* p) {
  const int* ks;
  const int nk = star_inst(p->ndim, p->rad, &ks);
  int bestK = ks[std::min(2, nk - 1)];
  const bool timed = !env_flag("STENCIL_MODEL_ONLY") && p->cells >= (size_t)1 << 16;
  float* tmp = nullptr;
  if (timed && hipMalloc(&tmp, p->cells * sizeof(float)) == hipSuccess) {
    launch_fill(tmp, p->cells, 0.5f, p->stream);
    launch_fill(p->scratch, p->cells, 0.5f, p->stream);
    StarCoef c{};
    c.c0 = 0.5f;
    for (int d = 0; d < p->rad; ++d) c.w[d] = c.e[d] = c.s[d] = c.n[d] = 0.125f / p->rad;
    p->star_cf = c;
    Star3Coef c3{};
    c3.c0 = 0.5f;
    for (int d = 0; d < p->rad; ++d) c3.w[d] = c3.e[d] = c3.s[d] = c3.n[d] = c3.b[d] = c3.a[d] = 0.25f / (3 * p->rad);
    p->star3_cf = c3;
    hipEvent_t e0, e1;
    hipEventCreate(&e0);
    hipEventCreate(&e1);
    auto time_k = [&](int K) -> double {
      stencil_plan_s q = *p;
      q.tuning.k = K;
      q.tuning.seg_len = pick_seg_star_nd(p, K);
      const double per_pass = (double)K * (double)p->cells;
      const int reps = std::max(2, std::min(192, (int)std::ceil(2.0e10 / per_pass)));
      run_star_pass(&q, K, K, tmp, p->scratch);
      hipEventRecord(e0, p->stream);
      for (int r = 0; r < reps; ++r) {
        const bool even = (r % 2) == 0;
        run_star_pass(&q, K, K, even ? p->scratch : tmp, even ? tmp : p->scratch);
      }
      hipEventRecord(e1, p->stream);
      hipEventSynchronize(e1);
      float ms = 0;
      hipEventElapsedTime(&ms, e0, e1);
      return ms > 0 ? reps * per_pass / (ms * 1e-3) : 0.0;
    };
    for (int w = 0; w < 2; ++w) time_k(ks[nk - 1]);
    std::vector<double> rate(nk, 0.0);
    for (int round = 0; round < 3; ++round)
      for (int i = 0; i < nk; ++i) rate[i] = std::max(rate[i], time_k(ks[i]));
    double best = 0;
    for (int i = 0; i < nk; ++i) {
      if (log_enabled())
        std::fprintf(stderr, "[stencil] tune star r=%d K=%d measured=%.1f GCell/s\n", p->rad, ks[i], rate[i] * 1e-9);
      if (rate[i] > best) {
        best = rate[i];
        bestK = ks[i];
      }
    }
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    hipStreamSynchronize(p->stream);
    hipFree(tmp);
  }
  hipGetLastError();
  p->tuning.variant = 2;
  p->tuning.k = bestK;
  p->tuning.seg_len = pick_seg_star_nd(p, bestK);
}

stencil_status_t set_device(const stencil_plan_s* p) {
  hipError_t e = hipSetDevice(p->device);
  if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
  return STENCIL_OK;
}

void destroy_side(stencil_plan_s* p) {
  if (p->side) {
    hipStreamSynchronize(p->side);
    hipStreamDestroy(p->side);
  }
  if (p->ev_fork) hipEventDestroy(p->ev_fork);
  if (p->ev_join) hipEventDestroy(p->ev_join);
  p->side = nullptr;
  p->ev_fork = p->ev_join = nullptr;
}

void free_ckpts(stencil_plan_s* p) {
  for (float* c : p->ckpts) hipFree(c);
  p->ckpts.clear();
  p->ckpt_every = 0;
  p->ckpt_T = -1;
}

// Forward with optional checkpoints; the work behind stencil_run and stencil_run_ckpt.
stencil_status_t forward(stencil_plan_s* p, float* grid, const float* power, const stencil_coeffs_t* coeffs, int T,
                         int ckpt_every, bool keep_ckpts) {
  if (!grid) return fail(STENCIL_ERR_INVALID_ARG, "grid is NULL");
  if (!coeffs) return fail(STENCIL_ERR_INVALID_ARG, "coeffs is NULL");
  if (T < 0) return fail(STENCIL_ERR_INVALID_ARG, "T must be >= 0");
  if (!coeffs_finite(*coeffs)) return fail(STENCIL_ERR_INVALID_ARG, "coefficients must be finite");
  if (p->form != STENCIL_DIFFUSION && !power) return fail(STENCIL_ERR_INVALID_ARG, "hotspot needs a power map");
  if ((reinterpret_cast<uintptr_t>(grid) & 3) || (power && (reinterpret_cast<uintptr_t>(power) & 3)))
    return fail(STENCIL_ERR_INVALID_ARG, "buffers must be 4-byte aligned");
  if (power == grid) return fail(STENCIL_ERR_INVALID_ARG, "power must not alias grid");
  stencil_status_t st = set_device(p);
  if (st != STENCIL_OK) return st;
  if (hipError_t e = poison_scratch(p); e != hipSuccess) return hip_fail(e, "poison fill");
  const KMode m = fwd_mode(p);
  const DevCoef cf = dev_coef(*coeffs, false, p->form == STENCIL_HOTSPOT_PHYS);
  const float* pw = (p->form != STENCIL_DIFFUSION) ? power : nullptr;
  int K;
  bool plain;
  resolve_k(p, m, &K, &plain);
  const int kpass = plain ? 1 : std::min(K, std::max(1, p->tuning.k));
  int counter = 0;
  if (!keep_ckpts) {
    return run_sequence(p, m, plain, K, split_steps(T, kpass), grid, grid, p->scratch, pw, nullptr, cf, &counter);
  }
  // checkpointed run: x_{j*ce} saved before segment j; each segment starts from its checkpoint
  if (ckpt_every <= 0) ckpt_every = std::max(1, (int)std::lround(std::sqrt((double)std::max(T, 1))));
  const int nck = T > 0 ? (T - 1) / ckpt_every + 1 : 0;
  if ((int)p->ckpts.size() != nck) free_ckpts(p);  // reuse the store when the count matches
  for (int j = (int)p->ckpts.size(); j < nck; ++j) {
    float* c = nullptr;
    hipError_t e = hipMalloc(&c, p->cells * sizeof(float));
    if (e != hipSuccess) {
      free_ckpts(p);
      hipGetLastError();
      return fail(STENCIL_ERR_OUT_OF_MEMORY, "checkpoint allocation failed");
    }
    p->ckpts.push_back(c);
  }
  p->ckpt_every = ckpt_every;
  p->ckpt_T = T;
  // x_0 is copied into checkpoint 0 once; segment j then runs from checkpoint j straight into
  // checkpoint j+1 (the last segment into grid), so no other checkpoint needs a copy
  if (nck > 0) {
    hipError_t e = hipMemcpyAsync(p->ckpts[0], grid, p->cells * sizeof(float), hipMemcpyDeviceToDevice, p->stream);
    if (e != hipSuccess) return hip_fail(e, "checkpoint copy");
  }
  for (int j = 0; j < nck; ++j) {
    const int seg_T = std::min(ckpt_every, T - j * ckpt_every);
    float* out = (j + 1 < nck) ? p->ckpts[j + 1] : grid;
    st = run_sequence(p, m, plain, K, split_steps(seg_T, kpass), p->ckpts[j], out, p->scratch, pw, nullptr, cf,
                      &counter);
    if (st != STENCIL_OK) return st;
  }
  return STENCIL_OK;
}

}  // namespace

// Device-side bitwise comparison used by the recompute check.
hipError_t launch_count_mismatch(const float* a, const float* b, size_t n, int* counter, hipStream_t s);

extern "C" {

const char* stencil_status_string(stencil_status_t s) {
  switch (s) {
    case STENCIL_OK: return "STENCIL_OK";
    case STENCIL_ERR_INVALID_ARG: return "STENCIL_ERR_INVALID_ARG";
    case STENCIL_ERR_UNSUPPORTED: return "STENCIL_ERR_UNSUPPORTED";
    case STENCIL_ERR_OUT_OF_MEMORY: return "STENCIL_ERR_OUT_OF_MEMORY";
    case STENCIL_ERR_HIP: return "STENCIL_ERR_HIP";
    case STENCIL_ERR_INTERNAL: return "STENCIL_ERR_INTERNAL";
  }
  return "STENCIL_ERR_UNKNOWN";
}

const char* stencil_last_error(void) { return g_last_error.c_str(); }

stencil_status_t stencil_create(stencil_plan_t* out, stencil_form_t form, int ndim, int nx, int ny, int nz,
                                const stencil_tuning_t* tuning, void* hip_stream) {
  if (!out) return fail(STENCIL_ERR_INVALID_ARG, "out is NULL");
  *out = nullptr;
  if (form != STENCIL_DIFFUSION && form != STENCIL_HOTSPOT && form != STENCIL_HOTSPOT_PHYS)
    return fail(STENCIL_ERR_INVALID_ARG, "unknown form");
  if (ndim != 2 && ndim != 3) return fail(STENCIL_ERR_INVALID_ARG, "ndim must be 2 or 3");
  if (form == STENCIL_HOTSPOT_PHYS && ndim != 2)
    return fail(STENCIL_ERR_UNSUPPORTED, "the physical hotspot form is defined for 2D grids");
  if (nx < 1 || ny < 1 || nz < 1) return fail(STENCIL_ERR_INVALID_ARG, "grid dimensions must be >= 1");
  if (ndim == 2 && nz != 1) return fail(STENCIL_ERR_INVALID_ARG, "2D grids need nz == 1");
  const double cells = (double)nx * ny * nz;
  if (cells > 9.0e18 / sizeof(float)) return fail(STENCIL_ERR_INVALID_ARG, "grid too large");
  if ((long)nx * ny > 0x7fffffffL && ndim == 3) return fail(STENCIL_ERR_UNSUPPORTED, "plane larger than 2^31 cells");
  if (tuning) {
    if (tuning->variant < 0 || tuning->variant > 2 || tuning->k < 0 || tuning->vec < 0 || tuning->bsize_x < 0 ||
        tuning->bsize_y < 0 || tuning->seg_len < 0 || tuning->nwork < 0)
      return fail(STENCIL_ERR_INVALID_ARG, "tuning fields must be >= 0 (variant 0..2)");
    if (tuning->nwork > 0 && ndim != 3)
      return fail(STENCIL_ERR_INVALID_ARG, "nwork selects the balanced launch of 3D grids");
    if (tuning->vec != 0 && tuning->vec != (ndim == 2 ? kTb2dV : kTb3dV))
      return fail(STENCIL_ERR_UNSUPPORTED, "vec is fixed by the kernel instantiation (2D: 4, 3D: 2)");
  }
  stencil_plan_s* p = new (std::nothrow) stencil_plan_s();
  if (!p) return fail(STENCIL_ERR_OUT_OF_MEMORY, "host allocation failed");
  p->form = form;
  p->ndim = ndim;
  p->nx = nx;
  p->ny = ny;
  p->nz = nz;
  p->cells = (size_t)nx * ny * nz;
  p->stream = reinterpret_cast<hipStream_t>(hip_stream);
  hipError_t e = hipGetDevice(&p->device);
  if (e != hipSuccess) {
    delete p;
    return hip_fail(e, "hipGetDevice");
  }
  e = hipMalloc(&p->scratch, p->cells * sizeof(float));
  if (e != hipSuccess) {
    delete p;
    hipGetLastError();
    return fail(STENCIL_ERR_OUT_OF_MEMORY, "scratch allocation failed");
  }
  if (ndim == 2) {
    // side stream (default priority) for the edge tiles of a 2D pass; without it every pass
    // runs as one launch
    if (hipStreamCreateWithFlags(&p->side, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&p->ev_fork, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&p->ev_join, hipEventDisableTiming) != hipSuccess) {
      destroy_side(p);
      hipGetLastError();
    }
  }
  stencil_tuning_t t{};
  if (tuning) t = *tuning;
  p->tuning = t;
  const KMode m = form_mode(form);
  if (t.variant == 1) {
    p->tuning.k = 1;
  } else if (t.k == 0 || t.seg_len == 0) {
    stencil_tuning_t tuned;
    if (t.k != 0) {
      // k fixed by the caller: only the segment length is chosen
      const int K = inst_k_for(ndim, m, std::min(t.k, tb_max_k(ndim, m)));
      tuned = t;
      tuned.k = std::min(t.k, tb_max_k(ndim, m));
      if (ndim == 2) {
        tuned.seg_len = pick_seg2d(K, nx, ny, 8);
      } else {
        // balanced launch, one workgroup per CU unless given; seg_len reports the planes of one
        // share
        p->nwork3d = t.nwork > 0 ? t.nwork : balanced_nwork3d(K, false, nx, ny, nz, 1);
        const Geom3D g = geom3d(K, false, nx, ny, nz, nz);
        tuned.seg_len = (int)ceil_div((long)g.ntx * g.nty * nz, p->nwork3d);
      }
    } else {
      TuneResult tr;
      stencil_status_t st = autotune(p, &tr);
      if (st != STENCIL_OK) {
        destroy_side(p);
        hipFree(p->scratch);
        delete p;
        return st;
      }
      tuned = tr.t;
      p->nwork3d = tr.nwork;
      p->adj_k = tr.adj_k;
      p->adj_seg = tr.adj_seg;
      p->adj_nwork = tr.adj_nwork;
      if (t.seg_len != 0) {
        // an explicit segment length selects the tile launch with that length
        tuned.seg_len = t.seg_len;
        p->nwork3d = 0;
        p->adj_seg = t.seg_len;
        p->adj_nwork = 0;
      }
      if (t.nwork > 0) p->nwork3d = t.nwork;  // an explicit balanced launch
    }
    p->tuning = tuned;
    p->tuning.variant = 2;
  } else {
    p->tuning.variant = 2;
    p->tuning.k = std::min(t.k, tb_max_k(ndim, m));
    if (ndim == 3 && t.nwork > 0) p->nwork3d = t.nwork;
  }
  // A caller-fixed k (or the plain variant) also fixes the adjoint's blocking: same k and
  // segment length, tile launch.
  if (p->adj_k == 0) {
    p->adj_k = p->tuning.k;
    p->adj_seg = p->tuning.seg_len;
    p->adj_nwork = 0;
  }
  if (log_enabled())
    std::fprintf(stderr, "[stencil] plan %dx%dx%d: forward k=%d seg=%d nwork=%d, adjoint k=%d seg=%d nwork=%d\n", nx,
                 ny, nz, p->tuning.k, p->tuning.seg_len, p->nwork3d, p->adj_k, p->adj_seg, p->adj_nwork);
  p->tuning.vec = ndim == 2 ? kTb2dV : kTb3dV;
  p->tuning.bsize_x = 64 * p->tuning.vec;
  p->tuning.bsize_y = ndim == 2 ? 0 : kTb3dWY;
  p->tuning.nwork = p->nwork3d;
  *out = p;
  return STENCIL_OK;
}

stencil_status_t stencil_get_tuning(stencil_plan_t plan, stencil_tuning_t* out) {
  if (!plan || !out) return fail(STENCIL_ERR_INVALID_ARG, "NULL argument");
  *out = plan->tuning;
  return STENCIL_OK;
}

stencil_status_t stencil_get_adjoint_tuning(stencil_plan_t p, stencil_tuning_t* out) {
  if (!p || !out) return fail(STENCIL_ERR_INVALID_ARG, "NULL argument");
  if (p->star) return fail(STENCIL_ERR_UNSUPPORTED, "no adjoint for radius-r star plans");
  stencil_tuning_t t = p->tuning;
  if (t.variant != 1) {
    const KMode m = p->form == STENCIL_HOTSPOT_PHYS ? KM_PHYS_ADJ_ACC : KM_ADJ_ACC;
    const int kreq = p->adj_k > 0 ? p->adj_k : std::max(1, p->tuning.k);
    t.k = std::min(kreq, tb_max_k(p->ndim, m));
    t.seg_len = p->adj_seg > 0 ? p->adj_seg : p->tuning.seg_len;
    t.nwork = p->adj_nwork;
    if (p->ndim == 3) t.bsize_y = kTb3dAdjWY;
  }
  *out = t;
  return STENCIL_OK;
}

stencil_status_t stencil_plan_model(stencil_plan_t p, int T, stencil_plan_model_t* out) {
  if (!p || !out) return fail(STENCIL_ERR_INVALID_ARG, "NULL argument");
  if (T < 0) return fail(STENCIL_ERR_INVALID_ARG, "T must be >= 0");
  if (p->star) {
    const int K = star_k_for(p->ndim, p->rad, std::max(1, p->tuning.k));
    const int kpass = std::min(K, std::max(1, p->tuning.k));
    ModelParts mp;
    stencil_plan_model_t r{};
    if (p->ndim == 3) {
      Geom3D g = geom_star3(p->rad, K, p->nx, p->ny, p->nz, p->tuning.seg_len);
      g.K = kpass;
      r.seconds = model_time_star3(g, p->rad, p->nx, p->ny, p->nz, T, &mp);
    } else {
      Geom2D g = geom_star(p->rad, K, p->nx, p->ny, p->tuning.seg_len);
      g.K = kpass;
      r.seconds = model_time_star(g, p->rad, p->nx, p->ny, T, &mp);
    }
    r.mem_seconds = mp.mem;
    r.alu_seconds = mp.alu;
    r.passes = (T + kpass - 1) / kpass;
    *out = r;
    return STENCIL_OK;
  }
  const KMode m = fwd_mode(p);
  const bool hot = p->form != STENCIL_DIFFUSION;
  int K;
  bool plain;
  resolve_k(p, m, &K, &plain);
  ModelParts mp;
  stencil_plan_model_t r{};
  if (plain) {
    // one step per launch: every step reads the grid (and power) and writes it once
    const DeviceInfo& d = device_info();
    const double bytes = (double)p->cells * 4.0 * ((hot ? 2 : 1) + 1);
    r.passes = T;
    r.mem_seconds = T * bytes / (d.hbm_gbs * 1e9 * d.achievable_frac);
    r.alu_seconds = 0.0;
    r.seconds = T * (bytes / (d.hbm_gbs * 1e9 * d.achievable_frac) + 4e-6);
  } else {
    const int kpass = std::min(K, std::max(1, p->tuning.k));
    if (p->ndim == 2) {
      Geom2D g = geom2d(K, p->nx, p->ny, p->tuning.seg_len);
      g.K = kpass;
      r.seconds = model_time_2d(g, p->nx, p->ny, T, hot, false, p->form == STENCIL_HOTSPOT_PHYS, &mp);
    } else if (p->nwork3d > 0) {
      Geom3D g = geom3d(K, false, p->nx, p->ny, p->nz, p->nz);
      g.K = kpass;
      r.seconds = model_time_3d_bal(g, p->nx, p->ny, p->nz, T, hot, false, p->nwork3d, &mp);
    } else {
      Geom3D g = geom3d(K, false, p->nx, p->ny, p->nz, p->tuning.seg_len);
      g.K = kpass;
      r.seconds = model_time_3d(g, p->nx, p->ny, p->nz, T, hot, false, &mp);
    }
    r.passes = (T + kpass - 1) / kpass;
    r.mem_seconds = mp.mem;
    r.alu_seconds = mp.alu;
  }
  *out = r;
  return STENCIL_OK;
}

void stencil_destroy(stencil_plan_t plan) {
  if (!plan) return;
  hipSetDevice(plan->device);
  hipStreamSynchronize(plan->stream);
  destroy_side(plan);
  free_ckpts(plan);
  hipFree(plan->scratch);
  hipFree(plan->verify_buf);
  hipFree(plan->mismatch);
  delete plan;
}

stencil_status_t stencil_run(stencil_plan_t plan, float* grid, const float* power, const stencil_coeffs_t* coeffs,
                             int T) {
  stencil_status_t st = check_plan(plan);
  if (st != STENCIL_OK) return st;
  if (plan->star) return fail(STENCIL_ERR_INVALID_ARG, "a radius-r star plan runs through stencil_run_star");
  return forward(plan, grid, power, coeffs, T, 0, false);
}

stencil_status_t stencil_run_ckpt(stencil_plan_t plan, float* grid, const float* power,
                                  const stencil_coeffs_t* coeffs, int T, int ckpt_every) {
  stencil_status_t st = check_plan(plan);
  if (st != STENCIL_OK) return st;
  if (plan->star) return fail(STENCIL_ERR_UNSUPPORTED, "checkpointed runs are not offered for radius-r star plans");
  if (ckpt_every < 0) return fail(STENCIL_ERR_INVALID_ARG, "ckpt_every must be >= 0");
  return forward(plan, grid, power, coeffs, T, ckpt_every, true);
}

stencil_status_t stencil_run_slab(stencil_plan_t p, const float* src, float* dst, const float* power,
                                  const stencil_coeffs_t* coeffs, int T, int ghost_lo, int ghost_hi) {
  stencil_status_t st = check_plan(p);
  if (st != STENCIL_OK) return st;
  if (p->star) return fail(STENCIL_ERR_UNSUPPORTED, "no slab pass for radius-r star plans");
  if (p->tuning.variant == 1) return fail(STENCIL_ERR_UNSUPPORTED, "the slab pass runs the temporal-blocked kernel");
  if (!src || !dst || !coeffs) return fail(STENCIL_ERR_INVALID_ARG, "src, dst and coeffs are required");
  if (src == dst) return fail(STENCIL_ERR_INVALID_ARG, "the slab pass is out of place: dst must not be src");
  if (p->form != STENCIL_DIFFUSION && !power) return fail(STENCIL_ERR_INVALID_ARG, "hotspot needs a power map");
  if (power && (power == dst)) return fail(STENCIL_ERR_INVALID_ARG, "power must not alias dst");
  if ((reinterpret_cast<uintptr_t>(src) | reinterpret_cast<uintptr_t>(dst) | reinterpret_cast<uintptr_t>(power)) & 3)
    return fail(STENCIL_ERR_INVALID_ARG, "buffers must be 4-byte aligned");
  if (!coeffs_finite(*coeffs)) return fail(STENCIL_ERR_INVALID_ARG, "coefficients must be finite");
  const int n = p->ndim == 2 ? p->ny : p->nz;  // cells along the streamed axis, ghosts included
  if (ghost_lo < 0 || ghost_hi < 0 || ghost_lo + ghost_hi >= n)
    return fail(STENCIL_ERR_INVALID_ARG, "ghost depths must be >= 0 and leave at least one interior plane");
  if (T < 0) return fail(STENCIL_ERR_INVALID_ARG, "T must be >= 0");
  if ((ghost_lo > 0 && T > ghost_lo) || (ghost_hi > 0 && T > ghost_hi))
    return fail(STENCIL_ERR_INVALID_ARG, "T exceeds a ghost depth: each step consumes one ghost plane per face");
  const KMode m = fwd_mode(p);
  if (T > tb_max_k(p->ndim, m))
    return fail(STENCIL_ERR_UNSUPPORTED, "T exceeds the largest fused step count of one pass (" +
                                             std::to_string(tb_max_k(p->ndim, m)) + ")");
  st = set_device(p);
  if (st != STENCIL_OK) return st;
  const size_t plane = p->ndim == 2 ? (size_t)p->nx : (size_t)p->nx * p->ny;
  const int lo = ghost_lo, hi = n - ghost_hi;
  if (T == 0) {
    hipError_t e = hipMemcpyAsync(dst + lo * plane, src + lo * plane, (size_t)(hi - lo) * plane * sizeof(float),
                                  hipMemcpyDeviceToDevice, p->stream);
    return e == hipSuccess ? STENCIL_OK : hip_fail(e, "hipMemcpyAsync");
  }
  const DevCoef cf = dev_coef(*coeffs, false, p->form == STENCIL_HOTSPOT_PHYS);
  const int K = inst_k_for(p->ndim, m, T);
  hipError_t e = run_pass(p, m, K, T, src, dst, p->form != STENCIL_DIFFUSION ? power : nullptr, nullptr, cf, lo, hi);
  return e == hipSuccess ? STENCIL_OK : hip_fail(e, "kernel launch");
}

stencil_status_t stencil_adjoint(stencil_plan_t p, const float* cot, const float* power,
                                 const stencil_coeffs_t* coeffs, int T, float* grad_x0, float* grad_power,
                                 int recompute) {
  stencil_status_t st = check_plan(p);
  if (st != STENCIL_OK) return st;
  if (p->star) return fail(STENCIL_ERR_UNSUPPORTED, "no adjoint for radius-r star plans");
  if (!cot || !grad_x0) return fail(STENCIL_ERR_INVALID_ARG, "cotangent and grad_x0 are required");
  if (!coeffs) return fail(STENCIL_ERR_INVALID_ARG, "coeffs is NULL");
  if (T < 0) return fail(STENCIL_ERR_INVALID_ARG, "T must be >= 0");
  if (!coeffs_finite(*coeffs)) return fail(STENCIL_ERR_INVALID_ARG, "coefficients must be finite");
  if (grad_x0 == cot || grad_power == cot || (grad_power && grad_power == grad_x0))
    return fail(STENCIL_ERR_INVALID_ARG, "outputs must not alias the cotangent or each other");
  if ((reinterpret_cast<uintptr_t>(cot) | reinterpret_cast<uintptr_t>(grad_x0) | reinterpret_cast<uintptr_t>(grad_power) |
       reinterpret_cast<uintptr_t>(power)) & 3)
    return fail(STENCIL_ERR_INVALID_ARG, "buffers must be 4-byte aligned");
  if (recompute != 0 && recompute != 1) return fail(STENCIL_ERR_INVALID_ARG, "recompute must be 0 or 1");
  if (recompute) {
    if (p->ckpt_T != T || p->ckpts.empty())
      return fail(STENCIL_ERR_INVALID_ARG, "recompute needs checkpoints of a stencil_run_ckpt with the same T");
    if (p->form != STENCIL_DIFFUSION && !power) return fail(STENCIL_ERR_INVALID_ARG, "recompute of hotspot needs power");
  }
  st = set_device(p);
  if (st != STENCIL_OK) return st;
  if (hipError_t e = poison_scratch(p); e != hipSuccess) return hip_fail(e, "poison fill");
  const bool hot = p->form != STENCIL_DIFFUSION;
  const bool phys = p->form == STENCIL_HOTSPOT_PHYS;
  float* gp = hot ? grad_power : nullptr;
  // The physical form's linear part is symmetric: its transposed step is the same formula
  // with no power and an ambient temperature of 0.
  KMode m = gp ? KM_ADJ_ACC : KM_ADJ;
  DevCoef cf = dev_coef(*coeffs, true);
  if (phys) {
    m = gp ? KM_PHYS_ADJ_ACC : KM_PHYS_ADJ;
    cf = dev_coef(*coeffs, false, true);
    cf.kamb = 0.0f;
  }
  if (gp) {
    hipError_t e = launch_fill(gp, p->cells, 0.0f, p->stream);
    if (e != hipSuccess) return hip_fail(e, "fill");
  } else if (grad_power) {
    hipError_t e = launch_fill(grad_power, p->cells, 0.0f, p->stream);
    if (e != hipSuccess) return hip_fail(e, "fill");
  }
  const bool plain = (p->tuning.variant == 1);
  const int kreq = p->adj_k > 0 ? p->adj_k : std::max(1, p->tuning.k);
  int K = inst_k_for(p->ndim, m, std::min(kreq, tb_max_k(p->ndim, m)));
  // the transposed passes run on the adjoint's own blocking
  stencil_plan_s qa = *p;
  qa.tuning.seg_len = p->adj_seg > 0 ? p->adj_seg : p->tuning.seg_len;
  qa.nwork3d = p->adj_nwork;
  const int kpass = plain ? 1 : K;
  int counter = 0;
  if (!recompute) {
    return run_sequence(&qa, m, plain, K, split_steps(T, kpass), cot, grad_x0, p->scratch, nullptr, gp, cf, &counter);
  }
  // Segment-wise reverse sweep: for segment j (last to first) recompute x from checkpoint j,
  // check it reproduces checkpoint j+1 bit for bit, then run the adjoint over the segment.
  if (!p->verify_buf) {
    hipError_t e = hipMalloc(&p->verify_buf, p->cells * sizeof(float));
    if (e != hipSuccess) return hip_fail(e, "hipMalloc");
    e = hipMalloc(&p->mismatch, sizeof(int));
    if (e != hipSuccess) return hip_fail(e, "hipMalloc");
  }
  hipError_t e = launch_fill_int(p->mismatch, 1, 0, p->stream);
  if (e != hipSuccess) return hip_fail(e, "fill");
  const int ce = p->ckpt_every;
  const int nck = (int)p->ckpts.size();
  const KMode fm = fwd_mode(p);
  const DevCoef fcf = dev_coef(*coeffs, false, phys);
  int Kf;
  bool plainf;
  resolve_k(p, fm, &Kf, &plainf);
  const int kfp = plainf ? 1 : std::min(Kf, std::max(1, p->tuning.k));
  const float* lam_src = cot;
  for (int j = nck - 1; j >= 0; --j) {
    const int seg_T = std::min(ce, T - j * ce);
    // recompute the segment into verify_buf (scratch is the ping-pong partner)
    st = run_sequence(p, fm, plainf, Kf, split_steps(seg_T, kfp), p->ckpts[j], p->verify_buf, p->scratch,
                      hot ? power : nullptr, nullptr, fcf, &counter);
    if (st != STENCIL_OK) return st;
    if (j + 1 < nck) {
      e = launch_count_mismatch(p->verify_buf, p->ckpts[j + 1], p->cells, p->mismatch, p->stream);
      if (e != hipSuccess) return hip_fail(e, "mismatch kernel");
    }
    // adjoint over this segment: lam_src -> grad_x0 (ping-pong partner scratch)
    st = run_sequence(&qa, m, plain, K, split_steps(seg_T, kpass), lam_src, grad_x0, p->scratch, nullptr, gp, cf,
                      &counter);
    if (st != STENCIL_OK) return st;
    lam_src = grad_x0;
  }
  if (nck == 0) {
    e = hipMemcpyAsync(grad_x0, cot, p->cells * sizeof(float), hipMemcpyDeviceToDevice, p->stream);
    if (e != hipSuccess) return hip_fail(e, "hipMemcpyAsync");
  }
  int mism = 0;
  e = hipMemcpyAsync(&mism, p->mismatch, sizeof(int), hipMemcpyDeviceToHost, p->stream);
  if (e != hipSuccess) return hip_fail(e, "hipMemcpyAsync");
  e = hipStreamSynchronize(p->stream);
  if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
  if (mism != 0)
    return fail(STENCIL_ERR_INTERNAL, "recomputed segment differs from stored checkpoint in " + std::to_string(mism) +
                                          " cells");
  return STENCIL_OK;
}

stencil_status_t stencil_model_estimate(const stencil_model_params_t* q, stencil_model_result_t* r) {
  if (!q || !r) return fail(STENCIL_ERR_INVALID_ARG, "NULL argument");
  if ((q->ndim != 2 && q->ndim != 3) || q->rad < 1 || q->par_vec < 1 || q->par_time < 1 || q->f_max_hz <= 0 ||
      q->size_cell < 1 || q->num_read < 0 || q->num_write < 0 || q->bsize_x < 1 || q->dim_x < 1 || q->dim_y < 1 ||
      q->iter < 0 || q->th_max_gbs <= 0 || (q->ndim == 3 && (q->bsize_y < 1 || q->dim_z < 1)))
    return fail(STENCIL_ERR_INVALID_ARG, "invalid model parameters");
  const double nacc = q->num_read + q->num_write;
  // Eq. 3
  r->th_mem_gbs = std::min(q->f_max_hz * q->par_vec * q->size_cell * nacc / 1e9, q->th_max_gbs);
  // Eq. 2, 4, 5
  const long halo = (long)q->rad * q->par_time;
  r->csize_x = q->bsize_x - 2 * halo;
  r->csize_y = q->ndim == 3 ? q->bsize_y - 2 * halo : 0;
  if (r->csize_x < 1 || (q->ndim == 3 && r->csize_y < 1))
    return fail(STENCIL_ERR_INVALID_ARG, "halo leaves an empty compute block");
  r->bnum_x = (q->dim_x + r->csize_x - 1) / r->csize_x;
  r->bnum_y = q->ndim == 3 ? (q->dim_y + r->csize_y - 1) / r->csize_y : 0;
  // Eq. 6 and 7: traversed cells per dimension minus the out-of-bound ones
  const double trav_x = (double)r->bnum_x * r->csize_x + 2.0 * halo;
  double size_input;
  if (q->ndim == 2) {
    r->t_cell = (double)r->bnum_x * q->bsize_x * q->dim_y;
    r->t_read = (r->t_cell - (trav_x - q->dim_x) * q->dim_y) * q->num_read;
    size_input = (double)q->dim_x * q->dim_y;
  } else {
    const double trav_y = (double)r->bnum_y * r->csize_y + 2.0 * halo;
    r->t_cell = (double)r->bnum_x * q->bsize_x * r->bnum_y * q->bsize_y * q->dim_z;
    r->t_read = ((double)r->bnum_x * q->bsize_x - (trav_x - q->dim_x)) *
                ((double)r->bnum_y * q->bsize_y - (trav_y - q->dim_y)) * q->dim_z * q->num_read;
    size_input = (double)q->dim_x * q->dim_y * q->dim_z;
  }
  r->t_write = size_input * q->num_write;
  // Eq. 8, 9
  const double passes = (double)((q->iter + q->par_time - 1) / q->par_time);
  r->run_time_s = passes * (r->t_read + r->t_write) * q->size_cell / (1e9 * r->th_mem_gbs);
  r->throughput_gbs = r->run_time_s > 0 ? nacc * size_input * q->size_cell * q->iter / (1e9 * r->run_time_s) : 0.0;
  return STENCIL_OK;
}

stencil_status_t stencil_create_star(stencil_plan_t* out, int ndim, int rad, int nx, int ny, int nz,
                                     const stencil_tuning_t* tuning, void* hip_stream) {
  if (!out) return fail(STENCIL_ERR_INVALID_ARG, "out is NULL");
  *out = nullptr;
  if (ndim != 2 && ndim != 3) return fail(STENCIL_ERR_INVALID_ARG, "ndim must be 2 or 3");
  if (rad < 1) return fail(STENCIL_ERR_INVALID_ARG, "rad must be >= 1");
  if (rad > kStarMaxR) return fail(STENCIL_ERR_UNSUPPORTED, "rad is at most 4 (the x-neighbours of a lane's 4 cells)");
  stencil_tuning_t t{};
  if (tuning) t = *tuning;
  if (t.variant < 0 || t.variant > 2 || t.k < 0 || t.vec < 0 || t.bsize_x < 0 || t.bsize_y < 0 || t.seg_len < 0 ||
      t.nwork != 0)
    return fail(STENCIL_ERR_INVALID_ARG, "tuning fields must be >= 0 (variant 0..2), nwork 0");
  if (t.vec != 0 && t.vec != kTb2dV) return fail(STENCIL_ERR_UNSUPPORTED, "vec is fixed at 4");
  // the plan itself (scratch, streams) without the radius-1 tuner: its blocking is set below
  stencil_tuning_t fixed{2, 1, 0, 0, 0, 1, 0};
  stencil_status_t st = stencil_create(out, STENCIL_DIFFUSION, ndim, nx, ny, nz, &fixed, hip_stream);
  if (st != STENCIL_OK) return st;
  stencil_plan_s* p = *out;
  p->star = true;
  p->rad = rad;
  const int* ks;
  const int nk = star_inst(ndim, rad, &ks);
  p->tuning = t;
  if (t.variant == 1) {
    p->tuning.k = 1;
    p->tuning.seg_len = t.seg_len > 0 ? t.seg_len : pick_seg_star_nd(p, 1);
  } else if (t.k > 0) {
    p->tuning.variant = 2;
    p->tuning.k = std::min(t.k, ks[nk - 1]);
    p->tuning.seg_len = t.seg_len > 0 ? t.seg_len : pick_seg_star_nd(p, star_k_for(ndim, rad, p->tuning.k));
  } else {
    star_tune(p);
  }
  if (ndim == 3) {
    p->tuning.vec = 1;
    p->tuning.bsize_x = p->tuning.bsize_y = kStar3W;
  } else {
    p->tuning.vec = kTb2dV;
    p->tuning.bsize_x = 64 * kTb2dV;
    p->tuning.bsize_y = 0;
  }
  p->tuning.nwork = 0;
  if (log_enabled())
    std::fprintf(stderr, "[stencil] star plan r=%d %dx%dx%d -> k=%d seg=%d\n", rad, nx, ny, nz, p->tuning.k,
                 p->tuning.seg_len);
  return STENCIL_OK;
}

// A radius-r star run of either form: power == nullptr is the diffusion form; otherwise the
// hotspot form with src = {cp, c_amb, t_amb}.
static stencil_status_t run_star(stencil_plan_t p, float* grid, const float* power, const float* weights, const float* src,
                          int T) {
  stencil_status_t st = check_plan(p);
  if (st != STENCIL_OK) return st;
  if (!p->star) return fail(STENCIL_ERR_INVALID_ARG, "not a radius-r star plan (stencil_create_star)");
  if (!grid || !weights) return fail(STENCIL_ERR_INVALID_ARG, "grid and weights are required");
  if (T < 0) return fail(STENCIL_ERR_INVALID_ARG, "T must be >= 0");
  if (reinterpret_cast<uintptr_t>(grid) & 3) return fail(STENCIL_ERR_INVALID_ARG, "grid must be 4-byte aligned");
  const int R = p->rad;
  const int nw = 1 + (p->ndim == 3 ? 6 : 4) * R;
  for (int i = 0; i < nw; ++i)
    if (!std::isfinite(weights[i])) return fail(STENCIL_ERR_INVALID_ARG, "weights must be finite");
  float cp = 0.0f, kamb = 0.0f;
  if (power) {
    if (!src) return fail(STENCIL_ERR_INVALID_ARG, "the hotspot form needs src = {cp, c_amb, t_amb}");
    for (int i = 0; i < 3; ++i)
      if (!std::isfinite(src[i])) return fail(STENCIL_ERR_INVALID_ARG, "src must be finite");
    if (reinterpret_cast<uintptr_t>(power) & 3) return fail(STENCIL_ERR_INVALID_ARG, "power must be 4-byte aligned");
    if (power == grid) return fail(STENCIL_ERR_INVALID_ARG, "power must not alias grid");
    cp = src[0];
    kamb = src[1] * src[2];  // rounded once in FP32
  }
  if (p->ndim == 3) {
    Star3Coef c{};
    c.c0 = weights[0];
    for (int d = 1; d <= R; ++d) {
      c.w[d - 1] = weights[2 * d - 1];
      c.e[d - 1] = weights[2 * d];
      c.s[d - 1] = weights[2 * R + d];
      c.n[d - 1] = weights[3 * R + d];
      c.b[d - 1] = weights[4 * R + d];
      c.a[d - 1] = weights[5 * R + d];
    }
    c.cp = cp;
    c.kamb = kamb;
    p->star3_cf = c;
  } else {
    StarCoef c{};
    c.c0 = weights[0];
    for (int d = 1; d <= R; ++d) {
      c.w[d - 1] = weights[2 * d - 1];
      c.e[d - 1] = weights[2 * d];
      c.s[d - 1] = weights[2 * R + d];
      c.n[d - 1] = weights[3 * R + d];
    }
    c.cp = cp;
    c.kamb = kamb;
    p->star_cf = c;
  }
  st = set_device(p);
  if (st != STENCIL_OK) return st;
  if (hipError_t e = poison_scratch(p); e != hipSuccess) return hip_fail(e, "poison fill");
  const int K = star_k_for(p->ndim, R, std::max(1, p->tuning.k));
  const int kpass = std::min(K, std::max(1, p->tuning.k));
  int counter = 0;
  p->star_power = power;
  st = run_sequence(p, KM_STAR, false, K, split_steps(T, kpass), grid, grid, p->scratch, nullptr, nullptr, DevCoef{},
                    &counter);
  p->star_power = nullptr;
  return st;
}

stencil_status_t stencil_run_star(stencil_plan_t p, float* grid, const float* weights, int T) {
  return run_star(p, grid, nullptr, weights, nullptr, T);
}

stencil_status_t stencil_run_star_hotspot(stencil_plan_t p, float* grid, const float* power, const float* weights,
                                          const float* src, int T) {
  if (!power) return fail(STENCIL_ERR_INVALID_ARG, "power is required");
  return run_star(p, grid, power, weights, src, T);
}

stencil_status_t stencil_adjoint_star(stencil_plan_t p, const float* cotangent, const float* weights,
                                      const float* src, int T, float* grad_x0, float* grad_power) {
  stencil_status_t st = check_plan(p);
  if (st != STENCIL_OK) return st;
  if (!p->star) return fail(STENCIL_ERR_INVALID_ARG, "not a radius-r star plan (stencil_create_star)");
  if (!cotangent || !grad_x0 || !weights) return fail(STENCIL_ERR_INVALID_ARG, "cotangent, grad_x0 and weights are required");
  if (T < 0) return fail(STENCIL_ERR_INVALID_ARG, "T must be >= 0");
  if ((reinterpret_cast<uintptr_t>(cotangent) | reinterpret_cast<uintptr_t>(grad_x0) |
       reinterpret_cast<uintptr_t>(grad_power)) & 3)
    return fail(STENCIL_ERR_INVALID_ARG, "buffers must be 4-byte aligned");
  if (grad_x0 == cotangent || (grad_power && (grad_power == cotangent || grad_power == grad_x0)))
    return fail(STENCIL_ERR_INVALID_ARG, "grad_x0 and grad_power must not alias cotangent or each other");
  if (grad_power && !src) return fail(STENCIL_ERR_INVALID_ARG, "grad_power needs src = {cp, c_amb, t_amb}");
  const int R = p->rad;
  const int nw = 1 + (p->ndim == 3 ? 6 : 4) * R;
  for (int i = 0; i < nw; ++i)
    if (!std::isfinite(weights[i])) return fail(STENCIL_ERR_INVALID_ARG, "weights must be finite");
  if (grad_power && !std::isfinite(src[0])) return fail(STENCIL_ERR_INVALID_ARG, "src must be finite");
  StarAdjArgs a{};
  a.nx = p->nx; a.ny = p->ny; a.nz = p->ndim == 3 ? p->nz : 1; a.ndim = p->ndim; a.rad = R;
  a.nbx = (p->nx + 255) / 256;
  a.stream = stream_stores(p);
  a.c0 = weights[0];
  a.cp = grad_power ? src[0] : 0.0f;
  for (int d = 1; d <= R; ++d) {
    a.wm[0][d - 1] = weights[2 * d - 1];  // x-d: w_d
    a.wp[0][d - 1] = weights[2 * d];      // x+d: e_d
    a.wp[1][d - 1] = weights[2 * R + d];  // y+d: s_d
    a.wm[1][d - 1] = weights[3 * R + d];  // y-d: n_d
    if (p->ndim == 3) {
      a.wm[2][d - 1] = weights[4 * R + d];  // z-d: b_d
      a.wp[2][d - 1] = weights[5 * R + d];  // z+d: a_d
    }
  }
  st = set_device(p);
  if (st != STENCIL_OK) return st;
  const size_t bytes = p->cells * sizeof(float);
  if (grad_power) {
    if (hipError_t e = launch_fill(grad_power, p->cells, 0.0f, p->stream); e != hipSuccess) return hip_fail(e, "fill");
  }
  if (T == 0) {
    hipError_t e = hipMemcpyAsync(grad_x0, cotangent, bytes, hipMemcpyDeviceToDevice, p->stream);
    return e == hipSuccess ? STENCIL_OK : hip_fail(e, "hipMemcpyAsync");
  }
  // lambda_T -> lambda_0, one launch per step, ping-pong between grad_x0 and plan scratch so
  // that the last step writes grad_x0
  const float* in = cotangent;
  for (int step = 1; step <= T; ++step) {
    float* out = ((T - step) % 2 == 0) ? grad_x0 : p->scratch;
    a.lam = in;
    a.out = out;
    a.gp = grad_power;
    if (hipError_t e = launch_star_adjoint(a, p->stream); e != hipSuccess) return hip_fail(e, "kernel launch");
    in = out;
  }
  return STENCIL_OK;
}

}  // extern "C"
