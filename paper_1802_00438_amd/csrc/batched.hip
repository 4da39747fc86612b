// batched.hip -- many grids of uneven sizes in one persistent launch per dimensionality.
//
// Every grid is split into temporal-blocked passes and overlapped tiles exactly as a single
// run would be (paper Sections 3.1-3.2).  All (grid, pass, tile) work items go into one list in
// pass-major order; resident workgroups claim items with an atomic counter and, before
// computing, wait until every tile of the previous pass of the same grid whose output
// overlaps the item's halo window has finished (a per-tile "passes done" flag, acquire/
// release at agent scope).  An item only ever waits for items that precede it in the list, so
// the claim order is a topological order and the launch cannot deadlock, whatever the number
// of resident workgroups.  Waiting on the previous-pass neighbours also covers the
// write-after-read hazard of the ping-pong buffers: the buffer a pass writes was last read by
// exactly those neighbours one pass earlier.
//
// Each grid uses an even number of passes (the steps spread over them), so its result ends in
// the caller's buffer.  The flag reset and both persistent kernels are captured once in a HIP
// graph and replayed; the reset is a fill kernel, not a memset node.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <utility>
#include <vector>
#include "runtime.hpp"

namespace {

constexpr int kBatchK2 = 16;  // fused-step capacity of the 2D persistent kernel
constexpr int kBatchK3 = 4;   // and of the 3D one
constexpr int kBatchR3 = tb3d_rows(kBatchK3, false), kBatchNW3 = tb3d_waves(kBatchK3, false);

struct BGrid {
  float* buf[2];  // buf[0] = caller's grid, buf[1] = scratch
  int nx, ny, nz;
  int cs, kr, ntx, seg, nseg;           // 2D geometry
  int csx, csy, krx, kry, nty, segz, nsegz;  // 3D geometry (ntx shared)
  int ax, ay, fx, fy;                         // 3D edge-flush tiling per axis
  int flag_off;
  int aligned;
  DevCoef cf;
};

struct BItem {
  int g, p, tile, keff;
};

// Every lane of the wave spins on the same flag with relaxed agent-scope loads; the loaded
// value is made wave-uniform (readfirstlane) so that the loop exit is a scalar branch.  One
// acquire fence after all of an item's waits (wait_neighbours) orders the item's reads after
// the producers' release stores.
__device__ __forceinline__ void wait_flag(const int* f, int want) {
  for (;;) {
    const int v = __builtin_amdgcn_readfirstlane(__hip_atomic_load(f, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
    if (v >= want) break;
    __builtin_amdgcn_s_sleep(2);
  }
}

// Claim the next work item for the whole workgroup, with no lane-divergent branch: every
// lane of the claiming wave issues the atomic (lane 0 adds 1, the others 0) and the result is
// taken from lane 0 with readfirstlane.  Divergent "if (threadIdx.x == 0)" blocks around the
// claim and the release would let the compiler restructure the persistent loop so that lane 0
// and lanes 1..63 run different loop nests; with the per-item control flow kept uniform, the
// loop is one scalar loop and every lane runs every trip.
__device__ __forceinline__ int wave_claim(int* counter) {
  const int lane = __lane_id();
  return __builtin_amdgcn_readfirstlane(atomicAdd(counter, lane == 0 ? 1 : 0));
}

__device__ __forceinline__ void wait_neighbours(const int* flags, int off, int tx, int ty, int ntx, int nty, int p) {
  if (p == 0) return;
  for (int dy = -1; dy <= 1; ++dy)
    for (int dx = -1; dx <= 1; ++dx) {
      const int x = tx + dx, y = ty + dy;
      if (x < 0 || y < 0 || x >= ntx || y >= nty) continue;
      wait_flag(flags + off + y * ntx + x, p);
    }
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
}

__global__ __launch_bounds__(64) void batched2d_kernel(const BGrid* __restrict__ grids, const BItem* __restrict__ items,
                                                       int nitems, int* counter, int* flags) {
  for (;;) {
    const int it = wave_claim(counter);
    if (it >= nitems) break;
    const BItem w = items[it];
    const BGrid& g = grids[w.g];
    const int tx = w.tile % g.ntx, ty = w.tile / g.ntx;
    wait_neighbours(flags, g.flag_off, tx, ty, g.ntx, g.nseg, w.p);
    Tb2dArgs a;
    a.src = g.buf[w.p & 1];
    a.dst = g.buf[(w.p + 1) & 1];
    a.power = nullptr;
    a.gp = nullptr;
    a.nx = g.nx; a.ny = g.ny; a.keff = w.keff;
    a.cs = g.cs; a.kr = g.kr; a.ntx = g.ntx; a.seg = g.seg; a.nseg = g.nseg;
    a.aligned = g.aligned;
    a.part = 0; a.ix0 = a.ix1 = a.iy0 = a.iy1 = 0;
    a.cf = g.cf;
    {
      Tb2dTile<kBatchK2, kTb2dV, false, false, false, false> t(a, threadIdx.x, nullptr);
      t.process(w.tile);
    }
    // all lanes publish the same flag value (release orders the wave's stores before it)
    st_release(flags + g.flag_off + w.tile, w.p + 1);
  }
}

__global__ __launch_bounds__(64 * kBatchNW3) void batched3d_kernel(const BGrid* __restrict__ grids,
                                                                 const BItem* __restrict__ items, int nitems,
                                                                 int* counter, int* flags) {
  __shared__ __align__(16) float hal[2 * kBatchK3 * kBatchNW3 * 2 * 64 * kTb3dV];
  __shared__ int sh;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  for (;;) {
    if (wave == 0) sh = wave_claim(counter);  // wave-uniform branch
    __syncthreads();
    const int it = __builtin_amdgcn_readfirstlane(sh);
    __syncthreads();
    if (it >= nitems) break;
    const BItem w = items[it];
    const BGrid& g = grids[w.g];
    const int tx = w.tile % g.ntx, rest = w.tile / g.ntx, ty = rest % g.nty, tz = rest / g.nty;
    if (w.p > 0) {
      for (int dz = -1; dz <= 1; ++dz) {
        const int z = tz + dz;
        if (z < 0 || z >= g.nsegz) continue;
        wait_neighbours(flags, g.flag_off + z * g.ntx * g.nty, tx, ty, g.ntx, g.nty, w.p);
      }
    }
    Tb3dArgs a;
    a.src = g.buf[w.p & 1];
    a.dst = g.buf[(w.p + 1) & 1];
    a.power = nullptr;
    a.gp = nullptr;
    a.nx = g.nx; a.ny = g.ny; a.nz = g.nz; a.keff = w.keff;
    a.csx = g.csx; a.csy = g.csy; a.krx = g.krx; a.kry = g.kry; a.ntx = g.ntx; a.nty = g.nty;
    a.segz = g.segz; a.nsegz = g.nsegz;
    a.nwork = 0;
    a.ax = g.ax; a.ay = g.ay; a.fx = g.fx; a.fy = g.fy;
    a.aligned = g.aligned;
    a.cf = g.cf;
    {
      Tb3dTile<kBatchK3, kTb3dV, kBatchR3, kBatchNW3, false, false, false, false> t(a, threadIdx.x & 63, threadIdx.x >> 6,
                                                                                 hal);
      t.process(w.tile);
    }
    __syncthreads();  // every wave's stores of this item precede wave 0's release
    if (wave == 0) st_release(flags + g.flag_off + w.tile, w.p + 1);
  }
}

__global__ void reset_kernel(int* flags, int nflags, int* counters) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < nflags) flags[i] = 0;
  if (i < 2) counters[i] = 0;
}

}  // namespace

struct stencil_batch_s {
  hipStream_t stream = nullptr;
  int device = 0;
  std::vector<stencil_batch_item_t> items;  // what was captured
  std::vector<float*> scratch;
  BGrid* d_grids = nullptr;
  BItem* d_items2 = nullptr;
  BItem* d_items3 = nullptr;
  int* d_flags = nullptr;
  int* d_counters = nullptr;
  int n2 = 0, n3 = 0, nflags = 0;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

using namespace stn;

namespace {

void release(stencil_batch_s* b) {
  if (!b) return;
  if (b->exec) hipGraphExecDestroy(b->exec);
  if (b->graph) hipGraphDestroy(b->graph);
  for (float* s : b->scratch) hipFree(s);
  hipFree(b->d_grids);
  hipFree(b->d_items2);
  hipFree(b->d_items3);
  hipFree(b->d_flags);
  hipFree(b->d_counters);
  delete b;
}

bool same_items(const stencil_batch_s* b, int n, const stencil_batch_item_t* items) {
  if ((int)b->items.size() != n) return false;
  for (int i = 0; i < n; ++i) {
    const stencil_batch_item_t& x = b->items[i];
    const stencil_batch_item_t& y = items[i];
    if (x.form != y.form || x.ndim != y.ndim || x.nx != y.nx || x.ny != y.ny || x.nz != y.nz || x.grid != y.grid ||
        x.T != y.T || std::memcmp(&x.coeffs, &y.coeffs, sizeof(x.coeffs)) != 0)
      return false;
  }
  return true;
}

// Steps of each pass: an even number of passes of at most kcap steps (0 passes when T == 0).
std::vector<int> even_split(int T, int kcap) {
  std::vector<int> v;
  if (T <= 0) return v;
  int P = (T + kcap - 1) / kcap;
  if (P % 2) ++P;
  const int base = T / P, rem = T % P;
  for (int i = 0; i < P; ++i) v.push_back(base + (i < rem ? 1 : 0));
  return v;
}

// The persistent 3D kernel keeps the uniform tiling (its tile decoding has no edge-flush case).
// Whether, along one axis, every tile's window reads only cells that its own tile and its two
// neighbours output: an item waits only for those neighbours of the previous pass.  Tile
// ranges follow the kernel's edge-flush tiling (flush = 1) or uniform tiling (flush = 0).
bool windows_within_neighbours(int n, int W, int nt, int f, int cs, int kr, bool flush) {
  auto range = [&](int t, int* o0, int* o1, int* w0) {
    if (!flush) {
      *o0 = t * cs; *o1 = std::min(*o0 + cs, n); *w0 = *o0 - kr;
    } else if (nt == 1) {
      *o0 = 0; *o1 = n; *w0 = 0;
    } else if (t == 0) {
      *o0 = 0; *o1 = f; *w0 = 0;
    } else if (t == nt - 1) {
      *o0 = std::max(f, n - f); *o1 = n; *w0 = n - W;
    } else {
      *o0 = f + (t - 1) * cs; *o1 = std::min(*o0 + cs, n - f); *w0 = *o0 - kr;
    }
  };
  for (int t = 0; t < nt; ++t) {
    int o0, o1, w0, lo0, lo1, lw, hi0, hi1, hw;
    range(t, &o0, &o1, &w0);
    range(std::max(t - 1, 0), &lo0, &lo1, &lw);
    range(std::min(t + 1, nt - 1), &hi0, &hi1, &hw);
    const int r0 = std::max(w0, 0), r1 = std::min(w0 + W, n);
    if (r0 < lo0 || r1 > hi1) return false;
  }
  return true;
}

// Geometry of a batched 3D grid: the kernel's edge-flush tiling where every window stays
// within its neighbours' outputs (the dependency rule of the work list), else uniform tiling
// on that axis.
Geom3D batch_geom3d(const BGrid& g, int segz) {
  Geom3D gg = geom3d(kBatchK3, false, g.nx, g.ny, g.nz, segz);
  const int WX = 64 * kTb3dV, WY = kTb3dWY;
  if (gg.ax && !windows_within_neighbours(g.nx, WX, gg.ntx, gg.fx, gg.csx, gg.krx, true)) {
    gg.ax = 0;
    gg.fx = 0;
    gg.ntx = (g.nx + gg.csx - 1) / gg.csx;
  }
  if (gg.ay && !windows_within_neighbours(g.ny, WY, gg.nty, gg.fy, gg.csy, gg.kry, true)) {
    gg.ay = 0;
    gg.fy = 0;
    gg.nty = (g.ny + gg.csy - 1) / gg.csy;
  }
  return gg;
}

// Work model of one work item: cell-levels it executes (its window times the streamed rows or
// planes, pipeline fill included, times the kernel's K levels).  Only ratios matter: it
// compares items of the same persistent kernel.
double item_work2d(const Geom2D& g) { return 64.0 * kTb2dV * (g.seg + 3.0 * kBatchK2) * kBatchK2; }
double item_work3d(const Geom3D& g) {
  return 64.0 * kTb3dV * kTb3dWY * (g.segz + 2.0 * kBatchK3 + 2.0) * kBatchK3;
}

// Segment length of every grid of one dimensionality.  A grid's passes form a chain of
// dependent steps: pass p of a tile waits for pass p-1 of its neighbours.  With `slots`
// resident workgroups the batch cannot finish before max(total work / slots, longest chain),
// so grids whose chain (passes x item time) exceeds the balanced share get shorter segments
// (shorter items, more halo work) until the chain fits, largest segment first.  Two
// refinement rounds, since shortening a chain adds work.
template <class GeomFn, class WorkFn>
std::vector<int> choose_segments(const std::vector<int>& idx, const std::vector<int>& passes,
                                 const std::vector<int>& len, const std::vector<int>& cands, double slots,
                                 GeomFn geom, WorkFn work) {
  std::vector<int> seg(passes.size(), 0);
  for (int i : idx) seg[i] = std::min(len[i], cands.front());
  for (int round = 0; round < 3; ++round) {
    double total = 0.0;
    for (int i : idx) {
      const auto g = geom(i, seg[i]);
      total += passes[i] * (double)g.first * work(g.second);
    }
    const double share = total / slots;
    for (int i : idx) {
      int pick = std::min(len[i], cands.back());
      for (int c : cands) {
        const int sgl = std::min(len[i], c);
        if (passes[i] * work(geom(i, sgl).second) <= share) {
          pick = sgl;
          break;
        }
      }
      seg[i] = pick;
    }
  }
  return seg;
}

stencil_status_t build(int n, const stencil_batch_item_t* items, hipStream_t stream, stencil_batch_s** out) {
  stencil_batch_s* b = new stencil_batch_s();
  b->stream = stream;
  hipGetDevice(&b->device);
  b->items.assign(items, items + n);
  std::vector<BGrid> grids(n);
  std::vector<std::vector<int>> steps(n);
  std::vector<int> ntiles(n), passes(n), len(n);
  std::vector<int> idx2, idx3;
  int nflags = 0;
  for (int i = 0; i < n; ++i) {
    const stencil_batch_item_t& it = items[i];
    BGrid& g = grids[i];
    std::memset(&g, 0, sizeof(g));
    g.nx = it.nx; g.ny = it.ny; g.nz = it.ndim == 3 ? it.nz : 1;
    g.cf = dev_coef(it.coeffs, false);
    const size_t cells = (size_t)g.nx * g.ny * g.nz;
    float* s = nullptr;
    if (hipMalloc(&s, cells * sizeof(float)) != hipSuccess) {
      hipGetLastError();
      release(b);
      return fail(STENCIL_ERR_OUT_OF_MEMORY, "batch scratch allocation failed");
    }
    b->scratch.push_back(s);
    g.buf[0] = it.grid;
    g.buf[1] = s;
    // The persistent kernels fuse up to kBatchK2 (2D) / kBatchK3 (3D) steps per pass, and a
    // pass costs the same for any number of fused steps up to that (levels past keff forward
    // their input), so each grid takes the fewest passes (even, so the result lands in its own
    // buffer), with the steps spread evenly over them.
    steps[i] = even_split(it.T, it.ndim == 2 ? kBatchK2 : kBatchK3);
    passes[i] = (int)steps[i].size();
    len[i] = it.ndim == 2 ? g.ny : g.nz;
    (it.ndim == 2 ? idx2 : idx3).push_back(i);
  }
  // resident workgroups of the two persistent kernels
  const DeviceInfo& d = device_info();
  int occ2 = 1, occ3 = 1;
  hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ2, batched2d_kernel, 64, 0);
  hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ3, batched3d_kernel, 64 * kBatchNW3, 0);
  const int slots2 = d.cus * std::max(1, occ2), slots3 = d.cus * std::max(1, occ3);
  auto geom2 = [&](int i, int sg) {
    const Geom2D gg = geom2d(kBatchK2, grids[i].nx, grids[i].ny, sg);
    return std::make_pair(gg.ntx * gg.nseg, gg);
  };
  auto geom3 = [&](int i, int sz) {
    const Geom3D gg = batch_geom3d(grids[i], sz);
    return std::make_pair(gg.ntx * gg.nty * gg.nsegz, gg);
  };
  const std::vector<int> seg2 = choose_segments(idx2, passes, len, {512, 384, 256, 192, 128, 96, 64, 48}, slots2,
                                                geom2, item_work2d);
  const std::vector<int> seg3 = choose_segments(idx3, passes, len, {64, 48, 32, 24, 16, 12, 8}, slots3, geom3,
                                                item_work3d);
  std::vector<double> t_item(n, 0.0);
  for (int i = 0; i < n; ++i) {
    BGrid& g = grids[i];
    if (items[i].ndim == 2) {
      const Geom2D gg = geom2d(kBatchK2, g.nx, g.ny, seg2[i]);
      g.cs = gg.cs; g.kr = gg.kr; g.ntx = gg.ntx; g.seg = gg.seg; g.nseg = gg.nseg;
      g.aligned = ((g.nx & 3) == 0) && ((reinterpret_cast<uintptr_t>(g.buf[0]) | reinterpret_cast<uintptr_t>(g.buf[1])) & 15) == 0;
      ntiles[i] = gg.ntx * gg.nseg;
      t_item[i] = item_work2d(gg);
    } else {
      const Geom3D gg = batch_geom3d(g, seg3[i]);
      g.csx = gg.csx; g.csy = gg.csy; g.krx = gg.krx; g.kry = gg.kry; g.ntx = gg.ntx; g.nty = gg.nty;
      g.segz = gg.segz; g.nsegz = gg.nsegz;
      g.ax = gg.ax; g.ay = gg.ay; g.fx = gg.fx; g.fy = gg.fy;
      g.aligned = ((g.nx & 1) == 0) && ((reinterpret_cast<uintptr_t>(g.buf[0]) | reinterpret_cast<uintptr_t>(g.buf[1])) & 7) == 0;
      ntiles[i] = gg.ntx * gg.nty * gg.nsegz;
      t_item[i] = item_work3d(gg);
    }
    g.flag_off = nflags;
    nflags += ntiles[i];
  }
  // Claim order: latest start time first (critical path priority).  Scheduled as late as
  // possible against the longest chain, pass p of grid g may start no later than
  // chain_max - (P_g - p) * t_g; sorting items by that bound starts the long chains first and
  // lets short grids fill in.  Pass p of a grid always sorts before its pass p+1, so the list
  // stays a topological order of the dependencies.
  struct Keyed {
    double lst;
    BItem it;
  };
  std::vector<Keyed> k2, k3;
  double chain2 = 0.0, chain3 = 0.0;
  for (int i = 0; i < n; ++i) (items[i].ndim == 2 ? chain2 : chain3) = std::max(
      items[i].ndim == 2 ? chain2 : chain3, passes[i] * t_item[i]);
  for (int i = 0; i < n; ++i) {
    const double chain = items[i].ndim == 2 ? chain2 : chain3;
    for (int p = 0; p < passes[i]; ++p) {
      const double lst = chain - (passes[i] - p) * t_item[i];
      for (int t = 0; t < ntiles[i]; ++t) (items[i].ndim == 2 ? k2 : k3).push_back({lst, {i, p, t, steps[i][p]}});
    }
  }
  auto order = [](const Keyed& x, const Keyed& y) {
    if (x.lst != y.lst) return x.lst < y.lst;
    if (x.it.g != y.it.g) return x.it.g < y.it.g;
    if (x.it.p != y.it.p) return x.it.p < y.it.p;
    return x.it.tile < y.it.tile;
  };
  std::stable_sort(k2.begin(), k2.end(), order);
  std::stable_sort(k3.begin(), k3.end(), order);
  std::vector<BItem> it2, it3;
  for (const Keyed& x : k2) it2.push_back(x.it);
  for (const Keyed& x : k3) it3.push_back(x.it);
  b->n2 = (int)it2.size();
  b->n3 = (int)it3.size();
  b->nflags = nflags;
  hipError_t e = hipSuccess;
  e = hipMalloc(&b->d_grids, sizeof(BGrid) * std::max(1, n));
  if (e == hipSuccess) e = hipMalloc(&b->d_items2, sizeof(BItem) * std::max(1, b->n2));
  if (e == hipSuccess) e = hipMalloc(&b->d_items3, sizeof(BItem) * std::max(1, b->n3));
  if (e == hipSuccess) e = hipMalloc(&b->d_flags, sizeof(int) * std::max(1, nflags));
  if (e == hipSuccess) e = hipMalloc(&b->d_counters, sizeof(int) * 2);
  if (e == hipSuccess && n) e = hipMemcpy(b->d_grids, grids.data(), sizeof(BGrid) * n, hipMemcpyHostToDevice);
  if (e == hipSuccess && b->n2) e = hipMemcpy(b->d_items2, it2.data(), sizeof(BItem) * b->n2, hipMemcpyHostToDevice);
  if (e == hipSuccess && b->n3) e = hipMemcpy(b->d_items3, it3.data(), sizeof(BItem) * b->n3, hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    stencil_status_t st = hip_fail(e, "batch setup");
    release(b);
    return st;
  }
  // persistent grid sizes: resident capacity of the device
  const int g2 = std::max(1, std::min(b->n2, slots2));
  const int g3 = std::max(1, std::min(b->n3, slots3));
  // capture: reset flags/counters, then the two persistent kernels
  hipStream_t cs = nullptr;
  e = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking);
  if (e == hipSuccess) e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
  if (e == hipSuccess) {
    const int nr = std::max(nflags, 2);
    hipLaunchKernelGGL(reset_kernel, dim3((nr + 255) / 256), dim3(256), 0, cs, b->d_flags, nflags, b->d_counters);
    if (b->n2)
      hipLaunchKernelGGL(batched2d_kernel, dim3(g2), dim3(64), 0, cs, b->d_grids, b->d_items2, b->n2, b->d_counters,
                         b->d_flags);
    if (b->n3)
      hipLaunchKernelGGL(batched3d_kernel, dim3(g3), dim3(64 * kBatchNW3), 0, cs, b->d_grids, b->d_items3, b->n3,
                         b->d_counters + 1, b->d_flags);
    e = hipStreamEndCapture(cs, &b->graph);
  }
  if (e == hipSuccess) e = hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0);
  if (cs) hipStreamDestroy(cs);
  if (e != hipSuccess) {
    stencil_status_t st = hip_fail(e, "graph capture");
    release(b);
    return st;
  }
  if (log_enabled()) {
    std::fprintf(stderr, "[stencil] batch: %d grids, %d 2D items (%d WGs), %d 3D items (%d WGs)\n", n, b->n2, g2,
                 b->n3, g3);
    for (int i = 0; i < n; ++i)
      std::fprintf(stderr, "[stencil]   grid %d: %dD %dx%dx%d T=%d passes=%d tiles=%d seg=%d\n", i, items[i].ndim,
                   items[i].nx, items[i].ny, items[i].nz, items[i].T, passes[i], ntiles[i],
                   items[i].ndim == 2 ? grids[i].seg : grids[i].segz);
  }
  *out = b;
  return STENCIL_OK;
}

}  // namespace

extern "C" {

stencil_status_t stencil_run_batched(int n, const stencil_batch_item_t* items, void* hip_stream,
                                     stencil_batch_t* graph_cache) {
  if (n < 0 || (n > 0 && !items)) return fail(STENCIL_ERR_INVALID_ARG, "invalid item list");
  for (int i = 0; i < n; ++i) {
    const stencil_batch_item_t& it = items[i];
    if (it.form != STENCIL_DIFFUSION)
      return fail(it.form == STENCIL_HOTSPOT || it.form == STENCIL_HOTSPOT_PHYS ? STENCIL_ERR_UNSUPPORTED
                                                                                : STENCIL_ERR_INVALID_ARG,
                  "batched launch supports the diffusion form");
    if ((it.ndim != 2 && it.ndim != 3) || it.nx < 1 || it.ny < 1 || it.nz < 1 || (it.ndim == 2 && it.nz != 1))
      return fail(STENCIL_ERR_INVALID_ARG, "item " + std::to_string(i) + ": bad dimensions");
    if (!it.grid || (reinterpret_cast<uintptr_t>(it.grid) & 3))
      return fail(STENCIL_ERR_INVALID_ARG, "item " + std::to_string(i) + ": grid NULL or misaligned");
    if (it.T < 0) return fail(STENCIL_ERR_INVALID_ARG, "item " + std::to_string(i) + ": T < 0");
    if (!coeffs_finite(it.coeffs)) return fail(STENCIL_ERR_INVALID_ARG, "item " + std::to_string(i) + ": coefficients");
    for (int j = 0; j < i; ++j)
      if (items[j].grid == it.grid) return fail(STENCIL_ERR_INVALID_ARG, "items share a grid");
  }
  hipStream_t s = reinterpret_cast<hipStream_t>(hip_stream);
  stencil_batch_s* b = nullptr;
  if (graph_cache && *graph_cache) {
    b = *graph_cache;
    if (!same_items(b, n, items))
      return fail(STENCIL_ERR_INVALID_ARG, "cached batch was built from different items");
  } else {
    stencil_status_t st = build(n, items, s, &b);
    if (st != STENCIL_OK) return st;
    if (graph_cache) *graph_cache = b;
  }
  hipError_t e = hipGraphLaunch(b->exec, s);
  if (e != hipSuccess) {
    stencil_status_t st = hip_fail(e, "hipGraphLaunch");
    if (!graph_cache) {
      hipStreamSynchronize(s);
      release(b);
    }
    return st;
  }
  if (!graph_cache) {
    e = hipStreamSynchronize(s);
    release(b);
    if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
  }
  return STENCIL_OK;
}

void stencil_batch_destroy(stencil_batch_t b) {
  if (!b) return;
  hipSetDevice(b->device);
  hipStreamSynchronize(b->stream);
  release(b);
}

}  // extern "C"
