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
// graph and replayed; the reset is a fill kernel, not a memset node.  In the graph the 2D and
// 3D kernels are parallel branches on a split of the CUs (see plan_batch); the no-allocation
// path runs them one after the other on the whole device.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
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

// Arguments of the persistent kernels.  err is a sticky flag (0 = no failure) that a wait
// sets when it gives up; spin_limit bounds the polls of one wait.
struct BLaunch {
  const BGrid* grids;
  const BItem* items;
  int nitems;
  int* counter;
  int* flags;
  int* err;
  int spin_limit;
};

// Every lane of the wave polls the same flag with relaxed agent-scope loads; the loaded value
// is made wave-uniform (readfirstlane) so that the loop exit is a scalar branch.  One acquire
// fence after all of an item's waits (wait_neighbours) orders the item's reads after the
// producers' release stores.  A wait is bounded: after spin_limit unsuccessful polls (about a
// microsecond each), or as soon as another wave has given up, it sets the sticky error flag
// and returns, so a scheduling fault ends the launch with an error instead of a hang (the
// item then runs on whatever its inputs hold; the host reports the error).
__device__ __forceinline__ void wait_flag(const int* f, int want, const BLaunch& L) {
  for (int n = 0;; ++n) {
    const int v = __builtin_amdgcn_readfirstlane(__hip_atomic_load(f, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
    if (v >= want) return;
    const int e = __builtin_amdgcn_readfirstlane(__hip_atomic_load(L.err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
    if (e != 0) return;
    if (n >= L.spin_limit) {
      __hip_atomic_store(L.err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      return;
    }
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

__device__ __forceinline__ void wait_neighbours(const BLaunch& L, int off, int tx, int ty, int ntx, int nty, int p) {
  if (p == 0) return;
  for (int dy = -1; dy <= 1; ++dy)
    for (int dx = -1; dx <= 1; ++dx) {
      const int x = tx + dx, y = ty + dy;
      if (x < 0 || y < 0 || x >= ntx || y >= nty) continue;
      wait_flag(L.flags + off + y * ntx + x, p, L);
    }
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
}

__global__ __launch_bounds__(64) void batched2d_kernel(BLaunch L) {
  for (;;) {
    const int it = wave_claim(L.counter);
    if (it >= L.nitems) break;
    const BItem w = L.items[it];
    const BGrid& g = L.grids[w.g];
    const int tx = w.tile % g.ntx, ty = w.tile / g.ntx;
    wait_neighbours(L, g.flag_off, tx, ty, g.ntx, g.nseg, w.p);
    Tb2dArgs a;
    a.src = g.buf[w.p & 1];
    a.dst = g.buf[(w.p + 1) & 1];
    a.power = nullptr;
    a.gp = nullptr;
    a.nx = g.nx; a.ny = g.ny; a.keff = w.keff;
    a.cs = g.cs; a.kr = g.kr; a.ntx = g.ntx; a.seg = g.seg; a.nseg = g.nseg;
    a.aligned = g.aligned;
    a.stream = 0;
    a.part = 0; a.ix0 = a.ix1 = a.iy0 = a.iy1 = 0;
    a.ylo = 0; a.yhi = g.ny;
    a.cf = g.cf;
    {
      Tb2dTile<kBatchK2, kTb2dV, false, false, false, false> t(a, threadIdx.x, nullptr);
      t.process(w.tile);
    }
    // all lanes publish the same flag value (release orders the wave's stores before it)
    st_release(L.flags + g.flag_off + w.tile, w.p + 1);
  }
}

__global__ __launch_bounds__(64 * kBatchNW3) void batched3d_kernel(BLaunch L) {
  __shared__ __align__(16) float hal[2 * kBatchK3 * kBatchNW3 * 2 * 64 * kTb3dV];
  __shared__ int sh;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  for (;;) {
    if (wave == 0) sh = wave_claim(L.counter);  // wave-uniform branch
    __syncthreads();
    const int it = __builtin_amdgcn_readfirstlane(sh);
    __syncthreads();
    if (it >= L.nitems) break;
    const BItem w = L.items[it];
    const BGrid& g = L.grids[w.g];
    const int tx = w.tile % g.ntx, rest = w.tile / g.ntx, ty = rest % g.nty, tz = rest / g.nty;
    if (w.p > 0) {
      for (int dz = -1; dz <= 1; ++dz) {
        const int z = tz + dz;
        if (z < 0 || z >= g.nsegz) continue;
        wait_neighbours(L, g.flag_off + z * g.ntx * g.nty, tx, ty, g.ntx, g.nty, w.p);
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
    a.zlo = 0; a.zhi = g.nz;
    a.cf = g.cf;
    {
      Tb3dTile<kBatchK3, kTb3dV, kBatchR3, kBatchNW3, false, false, false, false> t(a, threadIdx.x & 63, threadIdx.x >> 6,
                                                                                 hal);
      t.process(w.tile);
    }
    __syncthreads();  // every wave's stores of this item precede wave 0's release
    if (wave == 0) st_release(L.flags + g.flag_off + w.tile, w.p + 1);
  }
}

// Clears the pass flags and the two claim counters before a launch; clear_err also clears
// the error flag (counters[2]), which the graph path keeps sticky across replays.
__global__ void reset_kernel(int* flags, int nflags, int* counters, int clear_err) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < nflags) flags[i] = 0;
  if (i < 2 || (clear_err && i == 2)) counters[i] = 0;
}

constexpr size_t kNoAllocScratchBytes = size_t(8) << 20;

}  // namespace

// Scratch of the no-allocation launch (stencil_run_batched_noalloc): the grid table, the work
// lists, the pass flags and the counters of one batch, 8 MiB at most.  Each GPU the library
// runs on holds its own copy until the process ends.  Host code never uses this name as an
// address: the per-device address comes from hipGetSymbolAddress.
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

struct stencil_batch_s {
  hipStream_t stream = nullptr;
  int device = 0;
  std::vector<stencil_batch_item_t> items;  // what was captured
  std::vector<float*> scratch;
  void* d_mem = nullptr;  // grid table, work lists, flags and counters (layout of BLayout)
  size_t err_off = 0;       // byte offset of the error flag in d_mem
  int* err_host = nullptr;  // pinned copy of the error flag after the latest replay
  hipEvent_t done = nullptr;
  bool launched = false;
  int n2 = 0, n3 = 0, nflags = 0;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

using namespace stn;

namespace {

// Everything the persistent kernels need, planned on the host before it is placed in device
// memory (allocated by the graph path, the static scratch array by the no-allocation path).
struct BPlan {
  std::vector<BGrid> grids;
  std::vector<BItem> it2, it3;
  int nflags = 0;
  int g2 = 1, g3 = 1;  // persistent workgroups of the 2D and 3D launches
  bool concurrent = false;  // the two launches run side by side on disjoint CUs
  double w2 = 0.0, w3 = 0.0;  // modelled work of the two halves (item work units, summed)
  std::vector<int> passes, ntiles, seg;
};

// Byte offsets of the device tables of a plan, in one block.
struct BLayout {
  size_t grids, items2, items3, flags, counters, total;
};
size_t align256(size_t v) { return (v + 255) & ~size_t(255); }
BLayout layout_of(const BPlan& P) {
  BLayout L;
  L.grids = 0;
  L.items2 = align256(L.grids + sizeof(BGrid) * P.grids.size());
  L.items3 = align256(L.items2 + sizeof(BItem) * P.it2.size());
  L.flags = align256(L.items3 + sizeof(BItem) * P.it3.size());
  L.counters = align256(L.flags + sizeof(int) * (size_t)P.nflags);
  L.total = align256(L.counters + sizeof(int) * 4);
  return L;
}

// The host image of the tables (grid table, work lists; the flags and counters are cleared by
// the reset kernel), laid out as layout_of says, up to L.flags.
std::vector<unsigned char> table_image(const BPlan& P, const BLayout& L) {
  std::vector<unsigned char> img(L.flags, 0);
  if (!P.grids.empty()) std::memcpy(img.data() + L.grids, P.grids.data(), sizeof(BGrid) * P.grids.size());
  if (!P.it2.empty()) std::memcpy(img.data() + L.items2, P.it2.data(), sizeof(BItem) * P.it2.size());
  if (!P.it3.empty()) std::memcpy(img.data() + L.items3, P.it3.data(), sizeof(BItem) * P.it3.size());
  return img;
}

// Kernel arguments of the two persistent launches over tables based at `base`.
void launch_args(const BPlan& P, const BLayout& L, unsigned char* base, int spin_limit, BLaunch* a2, BLaunch* a3) {
  int* counters = reinterpret_cast<int*>(base + L.counters);
  int* flags = reinterpret_cast<int*>(base + L.flags);
  const BGrid* grids = reinterpret_cast<const BGrid*>(base + L.grids);
  *a2 = BLaunch{grids, reinterpret_cast<const BItem*>(base + L.items2), (int)P.it2.size(), counters, flags,
                counters + 2, spin_limit};
  *a3 = BLaunch{grids, reinterpret_cast<const BItem*>(base + L.items3), (int)P.it3.size(), counters + 1, flags,
                counters + 2, spin_limit};
}

// Polls one wait may make before it gives up (about a microsecond each, so tens of seconds):
// far longer than any dependency of a real batch.  STENCIL_DEBUG_SPIN_LIMIT overrides it, so
// tests can make every unsatisfied wait give up at once and check the error path.
int spin_limit() {
  const char* v = std::getenv("STENCIL_DEBUG_SPIN_LIMIT");
  if (v && *v) return std::max(0, std::atoi(v));
  return 1 << 25;
}

// Enqueue the reset and the two persistent kernels on stream s.  With a second stream s3 (and
// two events), the 3D kernel runs on s3 concurrently with the 2D kernel on s, forked after the
// reset and joined back into s.
hipError_t enqueue_launch(const BPlan& P, const BLayout& L, unsigned char* base, int clear_err, hipStream_t s,
                          hipStream_t s3 = nullptr, hipEvent_t fork = nullptr, hipEvent_t join = nullptr) {
  BLaunch a2, a3;
  launch_args(P, L, base, spin_limit(), &a2, &a3);
  const int nr = std::max(P.nflags, 3);
  hipLaunchKernelGGL(reset_kernel, dim3((nr + 255) / 256), dim3(256), 0, s, a2.flags, P.nflags,
                     reinterpret_cast<int*>(base + L.counters), clear_err);
  const bool both = !P.it2.empty() && !P.it3.empty() && s3 && fork && join;
  if (both) {
    hipError_t e = hipEventRecord(fork, s);
    if (e == hipSuccess) e = hipStreamWaitEvent(s3, fork, 0);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(batched3d_kernel, dim3(P.g3), dim3(64 * kBatchNW3), 0, s3, a3);
    hipLaunchKernelGGL(batched2d_kernel, dim3(P.g2), dim3(64), 0, s, a2);
    e = hipEventRecord(join, s3);
    if (e == hipSuccess) e = hipStreamWaitEvent(s, join, 0);
    if (e != hipSuccess) return e;
    return hipGetLastError();
  }
  if (!P.it2.empty()) hipLaunchKernelGGL(batched2d_kernel, dim3(P.g2), dim3(64), 0, s, a2);
  if (!P.it3.empty()) hipLaunchKernelGGL(batched3d_kernel, dim3(P.g3), dim3(64 * kBatchNW3), 0, s, a3);
  return hipGetLastError();
}

void release(stencil_batch_s* b) {
  if (!b) return;
  if (b->exec) hipGraphExecDestroy(b->exec);
  if (b->graph) hipGraphDestroy(b->graph);
  for (float* s : b->scratch) hipFree(s);
  hipFree(b->d_mem);
  if (b->err_host) hipHostFree(b->err_host);
  if (b->done) hipEventDestroy(b->done);
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
  if (gg.ax == 1 && !windows_within_neighbours(g.nx, WX, gg.ntx, gg.fx, gg.csx, gg.krx, true)) {
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

// Plan a batch: per-grid pass split and tiling, the flag offsets and the two work lists in
// claim order.  partners[i] is grid i's ping-pong partner (device, same size as the grid).
// concurrent: the launch may run the two halves side by side (the graph path).
BPlan plan_batch(int n, const stencil_batch_item_t* items, float* const* partners, bool concurrent) {
  BPlan P;
  P.grids.resize(n);
  std::vector<std::vector<int>> steps(n);
  P.ntiles.assign(n, 0);
  P.passes.assign(n, 0);
  P.seg.assign(n, 0);
  std::vector<int> len(n);
  std::vector<int> idx2, idx3;
  for (int i = 0; i < n; ++i) {
    const stencil_batch_item_t& it = items[i];
    BGrid& g = P.grids[i];
    std::memset(&g, 0, sizeof(g));
    g.nx = it.nx; g.ny = it.ny; g.nz = it.ndim == 3 ? it.nz : 1;
    g.cf = dev_coef(it.coeffs, false);
    g.buf[0] = it.grid;
    g.buf[1] = partners[i];
    // The persistent kernels fuse up to kBatchK2 (2D) / kBatchK3 (3D) steps per pass, and a
    // pass costs the same for any number of fused steps up to that (levels past keff forward
    // their input), so each grid takes the fewest passes (even, so the result lands in its own
    // buffer), with the steps spread evenly over them.
    steps[i] = even_split(it.T, it.ndim == 2 ? kBatchK2 : kBatchK3);
    P.passes[i] = (int)steps[i].size();
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
    const Geom2D gg = geom2d(kBatchK2, P.grids[i].nx, P.grids[i].ny, sg);
    return std::make_pair(gg.ntx * gg.nseg, gg);
  };
  auto geom3 = [&](int i, int sz) {
    const Geom3D gg = batch_geom3d(P.grids[i], sz);
    return std::make_pair(gg.ntx * gg.nty * gg.nsegz, gg);
  };
  const std::vector<int> seg2 = choose_segments(idx2, P.passes, len, {512, 384, 256, 192, 128, 96, 64, 48}, slots2,
                                                geom2, item_work2d);
  const std::vector<int> seg3 = choose_segments(idx3, P.passes, len, {64, 48, 32, 24, 16, 12, 8}, slots3, geom3,
                                                item_work3d);
  std::vector<double> t_item(n, 0.0);
  for (int i = 0; i < n; ++i) {
    BGrid& g = P.grids[i];
    if (items[i].ndim == 2) {
      const Geom2D gg = geom2d(kBatchK2, g.nx, g.ny, seg2[i]);
      g.cs = gg.cs; g.kr = gg.kr; g.ntx = gg.ntx; g.seg = gg.seg; g.nseg = gg.nseg;
      g.aligned = ((g.nx & 3) == 0) && ((reinterpret_cast<uintptr_t>(g.buf[0]) | reinterpret_cast<uintptr_t>(g.buf[1])) & 15) == 0;
      P.ntiles[i] = gg.ntx * gg.nseg;
      P.seg[i] = gg.seg;
      t_item[i] = item_work2d(gg);
    } else {
      const Geom3D gg = batch_geom3d(g, seg3[i]);
      g.csx = gg.csx; g.csy = gg.csy; g.krx = gg.krx; g.kry = gg.kry; g.ntx = gg.ntx; g.nty = gg.nty;
      g.segz = gg.segz; g.nsegz = gg.nsegz;
      g.ax = gg.ax; g.ay = gg.ay; g.fx = gg.fx; g.fy = gg.fy;
      g.aligned = ((g.nx & 1) == 0) && ((reinterpret_cast<uintptr_t>(g.buf[0]) | reinterpret_cast<uintptr_t>(g.buf[1])) & 7) == 0;
      P.ntiles[i] = gg.ntx * gg.nty * gg.nsegz;
      P.seg[i] = gg.segz;
      t_item[i] = item_work3d(gg);
    }
    g.flag_off = P.nflags;
    P.nflags += P.ntiles[i];
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
  for (int i = 0; i < n; ++i) {
    double& c = items[i].ndim == 2 ? chain2 : chain3;
    c = std::max(c, P.passes[i] * t_item[i]);
  }
  for (int i = 0; i < n; ++i) {
    const double chain = items[i].ndim == 2 ? chain2 : chain3;
    for (int p = 0; p < P.passes[i]; ++p) {
      const double lst = chain - (P.passes[i] - p) * t_item[i];
      for (int t = 0; t < P.ntiles[i]; ++t) (items[i].ndim == 2 ? k2 : k3).push_back({lst, {i, p, t, steps[i][p]}});
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
  for (const Keyed& x : k2) P.it2.push_back(x.it);
  for (const Keyed& x : k3) P.it3.push_back(x.it);
  for (const BItem& it : P.it2) P.w2 += t_item[it.g];
  for (const BItem& it : P.it3) P.w3 += t_item[it.g];
  // Persistent grid sizes: the resident capacity of the device.  With both dimensionalities
  // and `concurrent`, the two launches run side by side on a split of the CUs (a 3D
  // workgroup takes a whole CU's registers, so the halves cannot share a CU): the 3D half
  // gets the share kappa*w3 / (w2 + kappa*w3) of the CUs, clamped to [1/8, 7/8].  kappa = 2.4,
  // the cost of a 3D item-work unit relative to a 2D one per CU, is the ratio at which the
  // split met the measured optimum on the 64-grid batch (160 of 256 CUs: 39.8 ms, against
  // 41.8 / 40.7 / 44.4 / 45.6 ms at 144 / 152 / 168 / 176 CUs and 45.1 ms back to back).
  // STENCIL_BATCH_SPLIT sets the 3D CUs instead (0: back to back).
  P.g2 = std::max(1, std::min((int)P.it2.size(), slots2));
  P.g3 = std::max(1, std::min((int)P.it3.size(), slots3));
  if (concurrent && !P.it2.empty() && !P.it3.empty()) {
    constexpr double kappa = 2.4;
    int c3 = (int)std::lround(d.cus * kappa * P.w3 / (P.w2 + kappa * P.w3));
    c3 = std::max(d.cus / 8, std::min(d.cus - d.cus / 8, c3));
    const char* sp = std::getenv("STENCIL_BATCH_SPLIT");
    if (sp && *sp) c3 = std::max(0, std::min(d.cus - 1, std::atoi(sp)));
    if (c3 > 0) {
      P.g3 = std::max(1, std::min((int)P.it3.size(), c3 * std::max(1, occ3)));
      P.g2 = std::max(1, std::min((int)P.it2.size(), (d.cus - c3) * std::max(1, occ2)));
      P.concurrent = true;
    }
  }
  return P;
}

void log_plan(int n, const stencil_batch_item_t* items, const BPlan& P, const char* how) {
  if (!log_enabled()) return;
  std::fprintf(stderr, "[stencil] batch (%s): %d grids, %zu 2D items (%d WGs), %zu 3D items (%d WGs), work %.4g / %.4g%s\n",
               how, n, P.it2.size(), P.g2, P.it3.size(), P.g3, P.w2, P.w3, P.concurrent ? ", concurrent" : "");
  for (int i = 0; i < n; ++i)
    std::fprintf(stderr, "[stencil]   grid %d: %dD %dx%dx%d T=%d passes=%d tiles=%d seg=%d\n", i, items[i].ndim,
                 items[i].nx, items[i].ny, items[i].nz, items[i].T, P.passes[i], P.ntiles[i], P.seg[i]);
}

// Graph path: plan-owned partner grids and tables, captured once.
stencil_status_t build(int n, const stencil_batch_item_t* items, hipStream_t stream, stencil_batch_s** out) {
  stencil_batch_s* b = new stencil_batch_s();
  b->stream = stream;
  hipGetDevice(&b->device);
  b->items.assign(items, items + n);
  for (int i = 0; i < n; ++i) {
    const stencil_batch_item_t& it = items[i];
    const size_t cells = (size_t)it.nx * it.ny * (it.ndim == 3 ? it.nz : 1);
    float* s = nullptr;
    if (hipMalloc(&s, cells * sizeof(float)) != hipSuccess) {
      hipGetLastError();
      release(b);
      return fail(STENCIL_ERR_OUT_OF_MEMORY, "batch scratch allocation failed");
    }
    b->scratch.push_back(s);
  }
  const BPlan P = plan_batch(n, items, b->scratch.data(), true);
  const BLayout L = layout_of(P);
  b->n2 = (int)P.it2.size();
  b->n3 = (int)P.it3.size();
  b->nflags = P.nflags;
  b->err_off = L.counters + 2 * sizeof(int);
  const std::vector<unsigned char> img = table_image(P, L);
  hipError_t e = hipMalloc(&b->d_mem, L.total);
  if (e == hipSuccess) e = hipHostMalloc(reinterpret_cast<void**>(&b->err_host), sizeof(int));
  if (e == hipSuccess) e = hipEventCreateWithFlags(&b->done, hipEventDisableTiming);
  if (e == hipSuccess && !img.empty()) e = hipMemcpy(b->d_mem, img.data(), img.size(), hipMemcpyHostToDevice);
  // the error flag is cleared once here and stays set across replays once a wait gives up
  unsigned char* base = static_cast<unsigned char*>(b->d_mem);
  if (e == hipSuccess) e = launch_fill_int(reinterpret_cast<int*>(base + L.counters), 4, 0, stream);
  if (e == hipSuccess) e = hipStreamSynchronize(stream);
  if (e != hipSuccess) {
    stencil_status_t st = hip_fail(e, "batch setup");
    release(b);
    return st;
  }
  if (b->err_host) *b->err_host = 0;
  // capture: reset flags/counters, then the two persistent kernels
  hipStream_t cs = nullptr, cs3 = nullptr;
  hipEvent_t fork = nullptr, join = nullptr;
  e = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking);
  if (e == hipSuccess && P.concurrent) {
    e = hipStreamCreateWithFlags(&cs3, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&fork, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&join, hipEventDisableTiming);
  }
  if (e == hipSuccess) e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
  if (e == hipSuccess) {
    const hipError_t le = enqueue_launch(P, L, base, 0, cs, cs3, fork, join);
    e = hipStreamEndCapture(cs, &b->graph);
    if (e == hipSuccess) e = le;
  }
  if (e == hipSuccess) e = hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0);
  if (fork) hipEventDestroy(fork);
  if (join) hipEventDestroy(join);
  if (cs3) hipStreamDestroy(cs3);
  if (cs) hipStreamDestroy(cs);
  if (e != hipSuccess) {
    stencil_status_t st = hip_fail(e, "graph capture");
    release(b);
    return st;
  }
  log_plan(n, items, P, "graph");
  *out = b;
  return STENCIL_OK;
}

stencil_status_t check_items(int n, const stencil_batch_item_t* items) {
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
  return STENCIL_OK;
}

// Error of the latest replay of b that has completed, if any (non-blocking).
stencil_status_t replay_status(stencil_batch_s* b, bool wait) {
  if (!b->launched) return STENCIL_OK;
  if (wait) {
    hipError_t e = hipEventSynchronize(b->done);
    if (e != hipSuccess) return hip_fail(e, "hipEventSynchronize");
  } else if (hipEventQuery(b->done) != hipSuccess) {
    hipGetLastError();  // hipErrorNotReady: the latest replay is still running
    return STENCIL_OK;
  }
  if (*b->err_host)
    return fail(STENCIL_ERR_INTERNAL, "a dependency wait of the batched launch exceeded its bound (the results are invalid)");
  return STENCIL_OK;
}

// Per-device state of the no-allocation launch: the address of this device's copy of
// `scratch`, looked up once with the device current, and a lock that serialises the calls of
// this process on the device (they share the array).
struct NoAllocDev {
  std::mutex mu;
  bool ready = false;
  unsigned char* ptr = nullptr;
};
constexpr int kMaxDevices = 64;
NoAllocDev g_noalloc[kMaxDevices];

}  // namespace

extern "C" {

stencil_status_t stencil_run_batched(int n, const stencil_batch_item_t* items, void* hip_stream,
                                     stencil_batch_t* graph_cache) {
  stencil_status_t st = check_items(n, items);
  if (st != STENCIL_OK) return st;
  hipStream_t s = reinterpret_cast<hipStream_t>(hip_stream);
  stencil_batch_s* b = nullptr;
  if (graph_cache && *graph_cache) {
    b = *graph_cache;
    if (!same_items(b, n, items))
      return fail(STENCIL_ERR_INVALID_ARG, "cached batch was built from different items");
    st = replay_status(b, false);
    if (st != STENCIL_OK) return st;
  } else {
    st = build(n, items, s, &b);
    if (st != STENCIL_OK) return st;
    if (graph_cache) *graph_cache = b;
  }
  hipError_t e = hipGraphLaunch(b->exec, s);
  // the error flag of this replay goes to pinned host memory, read once the replay is done
  if (e == hipSuccess)
    e = hipMemcpyAsync(b->err_host, static_cast<unsigned char*>(b->d_mem) + b->err_off, sizeof(int),
                       hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipEventRecord(b->done, s);
  if (e != hipSuccess) {
    st = hip_fail(e, "hipGraphLaunch");
    if (!graph_cache) {
      hipStreamSynchronize(s);
      release(b);
    }
    return st;
  }
  b->launched = true;
  if (!graph_cache) {
    st = replay_status(b, true);
    release(b);
    return st;
  }
  return STENCIL_OK;
}

stencil_status_t stencil_batch_sync(stencil_batch_t b) {
  if (!b) return fail(STENCIL_ERR_INVALID_ARG, "batch is NULL");
  hipError_t e = hipSetDevice(b->device);
  if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
  return replay_status(b, true);
}

void stencil_batch_destroy(stencil_batch_t b) {
  if (!b) return;
  hipSetDevice(b->device);
  hipStreamSynchronize(b->stream);
  release(b);
}

stencil_status_t stencil_run_batched_noalloc(int n, const stencil_batch_item_t* items, float* const* partners,
                                             void* hip_stream) {
  stencil_status_t st = check_items(n, items);
  if (st != STENCIL_OK) return st;
  if (n > 0 && !partners) return fail(STENCIL_ERR_INVALID_ARG, "partners is NULL");
  for (int i = 0; i < n; ++i) {
    if (!partners[i] || (reinterpret_cast<uintptr_t>(partners[i]) & 3))
      return fail(STENCIL_ERR_INVALID_ARG, "partner " + std::to_string(i) + ": NULL or misaligned");
    for (int j = 0; j < n; ++j)
      if (partners[i] == items[j].grid || (j < i && partners[j] == partners[i]))
        return fail(STENCIL_ERR_INVALID_ARG, "partner " + std::to_string(i) + " aliases another buffer");
  }
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  if (dev < 0 || dev >= kMaxDevices) return fail(STENCIL_ERR_UNSUPPORTED, "device index beyond 63");
  NoAllocDev& D = g_noalloc[dev];
  std::lock_guard<std::mutex> lk(D.mu);
  if (!D.ready) {
    // this device's copy of the scratch array, looked up with the device current
    void* ptr = nullptr;
    e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr) return hip_fail(e != hipSuccess ? e : hipErrorInvalidSymbol, "hipGetSymbolAddress");
    D.ptr = static_cast<unsigned char*>(ptr);
    D.ready = true;
  }
  if (n == 0) return STENCIL_OK;
  hipStream_t s = reinterpret_cast<hipStream_t>(hip_stream);
  const BPlan P = plan_batch(n, items, partners, false);
  const BLayout L = layout_of(P);
  if (L.total > kNoAllocScratchBytes)
    return fail(STENCIL_ERR_INVALID_ARG, "the batch needs " + std::to_string(L.total) +
                                             " bytes of tables; the no-allocation launch holds at most " +
                                             std::to_string(kNoAllocScratchBytes));
  const std::vector<unsigned char> img = table_image(P, L);
  int err = 0;
  if (!img.empty()) e = hipMemcpyAsync(D.ptr, img.data(), img.size(), hipMemcpyHostToDevice, s);
  // the reset clears the flags, the claim counters and the error flag left by the last call
  if (e == hipSuccess) e = enqueue_launch(P, L, D.ptr, 1, s);
  if (e == hipSuccess)
    e = hipMemcpyAsync(&err, D.ptr + L.counters + 2 * sizeof(int), sizeof(int), hipMemcpyDeviceToHost, s);
  // synchronous, like the uncached stencil_run_batched: the host tables and the error flag
  // are read before the call returns
  const hipError_t es = hipStreamSynchronize(s);
  if (e == hipSuccess) e = es;
  if (e != hipSuccess) return hip_fail(e, "batched launch");
  log_plan(n, items, P, "no allocation");
  if (err) return fail(STENCIL_ERR_INTERNAL, "a dependency wait of the batched launch exceeded its bound (the results are invalid)");
  return STENCIL_OK;
}

}  // extern "C"
