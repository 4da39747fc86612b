// launch.hpp -- internal interface between the host runtime and the kernel translation units.
#pragma once
#include <hip/hip_runtime.h>
#include "tb2d.hpp"
#include "tb3d.hpp"
#include "plain.hpp"
#include "star2d.hpp"
#include "star3d.hpp"
#include "star_adjoint.hpp"

// Kernel mode: forward diffusion, forward hotspot, transposed step (adjoint) without / with
// grad_p accumulation, or the forward step of Table 2's physical Hotspot 2D formula (2D only).
enum KMode {
  KM_DIFF = 0, KM_HOT = 1, KM_ADJ = 2, KM_ADJ_ACC = 3, KM_PHYS = 4, KM_STAR = 5,
  KM_PHYS_ADJ = 6, KM_PHYS_ADJ_ACC = 7  // transposed step of the physical form, without / with grad_p
};

// Tile shapes of the temporal-blocked kernels.
// 3D windows: 128 x 48 cells forward, 128 x 32 for the transposed (adjoint) step.  The
// forward window is split over the workgroup's waves as 16 waves of 3 rows (1024 threads, four
// waves per SIMD) where the K-level state fits in 128 VGPRs and the halo rows in LDS, else as
// 8 waves of 6 rows (two waves per SIMD).  Both splits give the same tiles.
constexpr int kTb3dV = 2, kTb3dWY = 48, kTb3dAdjWY = 32;
constexpr int kTb3dAdjR = 2, kTb3dAdjNW = 16;
constexpr int tb3d_rows(int K, bool hot) { return (hot ? K <= 3 : K <= 4) ? 3 : 6; }
constexpr int tb3d_waves(int K, bool hot) { return kTb3dWY / tb3d_rows(K, hot); }

// Largest fused-step count instantiated per (dimensionality, mode); every k in
// [1, max] is served by the smallest instantiated K >= k (levels past k forward their input).
int tb_max_k(int ndim, KMode m);
// Instantiated K values (ascending) for (ndim, mode); returns the count.
int tb_instantiated(int ndim, KMode m, const int** ks);

hipError_t launch_tb2d(int K, KMode m, bool full, const Tb2dArgs& a, hipStream_t s);
hipError_t launch_tb3d(int K, KMode m, bool full, const Tb3dArgs& a, hipStream_t s);
hipError_t launch_plain(KMode m, const PlainArgs& a, hipStream_t s);
hipError_t launch_fill(float* p, size_t n, float v, hipStream_t s);
// Radius-r 2D star kernels (star2d.hpp): instantiated K values (ascending) for radius R, and
// the launch of one pass.
int star_instantiated(int R, const int** ks);
hipError_t launch_star2d(int R, int K, const Star2dArgs& a, hipStream_t s);
// Radius-r 3D star kernels (star3d.hpp): the same for 3D.
int star3_instantiated(int R, const int** ks);
hipError_t launch_star3d(int R, int K, const Star3dArgs& a, hipStream_t s);
// One transposed step of a radius-r star stencil (star_adjoint.hpp).
hipError_t launch_star_adjoint(const StarAdjArgs& a, hipStream_t s);
hipError_t launch_fill_int(int* p, size_t n, int v, hipStream_t s);

// Per-mode launchers (one translation unit each).
hipError_t launch_tb2d_diff(int K, bool full, const Tb2dArgs& a, hipStream_t s);
hipError_t launch_tb2d_hot(int K, bool full, const Tb2dArgs& a, hipStream_t s);
hipError_t launch_tb2d_adj(int K, bool acc, bool full, const Tb2dArgs& a, hipStream_t s);
hipError_t launch_tb2d_phys(int K, bool full, const Tb2dArgs& a, hipStream_t s);
hipError_t launch_tb2d_phys_adj(int K, bool acc, bool full, const Tb2dArgs& a, hipStream_t s);
hipError_t launch_tb3d_diff(int K, bool full, const Tb3dArgs& a, hipStream_t s);
hipError_t launch_tb3d_hot(int K, bool full, const Tb3dArgs& a, hipStream_t s);
hipError_t launch_tb3d_adj(int K, bool acc, bool full, const Tb3dArgs& a, hipStream_t s);

// One input plane in flight per workgroup: a second one (PD = 2) measured no faster for
// diffusion and 27% slower for the K = 2 hotspot pass.
#define TB3D_PD(K, HOT, ADJ) 1
#define TB_LAUNCH3D(K, R, NW, HOT, ADJ, ACC, FULL, a, s)                                               \
  do {                                                                                                  \
    hipLaunchKernelGGL((tb3d_kernel<K, kTb3dV, R, NW, HOT, ADJ, ACC, FULL, TB3D_PD(K, HOT, ADJ)>),     \
                       dim3((a).nwork > 0 ? (a).nwork : (a).ntx * (a).nty * (a).nsegz), dim3(64 * NW), 0, s, a); \
    return hipGetLastError();                                                                           \
  } while (0)
