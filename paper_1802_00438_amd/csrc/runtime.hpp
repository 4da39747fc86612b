// runtime.hpp -- host-side internals shared by the runtime translation units.
#pragma once
#include <hip/hip_runtime.h>
#include <string>
#include <vector>
#include "../../include/stencil.h"
#include "launch.hpp"

namespace stn {

// Thread-local error detail behind stencil_last_error().
void set_error(const std::string& msg);
stencil_status_t fail(stencil_status_t st, const std::string& msg);
stencil_status_t hip_fail(hipError_t e, const char* what);
bool env_flag(const char* name);
bool log_enabled();

// Device facts used by the cost model (queried once, with published MI355X fallbacks).
struct DeviceInfo {
  int cus = 256;
  double hbm_gbs = 8000.0;      // peak HBM3E bandwidth
  double achievable_frac = 0.72;
  double valu_lane_ops = 256.0 * 4 * 16 * 2.4e9;  // CUs x SIMDs x lanes x clock (non-packed FP32)
};
const DeviceInfo& device_info();

// Geometry of one temporal-blocked pass (fixed by the instantiated K and the grid).
struct Geom2D {
  int K = 0, cs = 0, kr = 0, ntx = 0, seg = 0, nseg = 0;
};
struct Geom3D {
  int K = 0, csx = 0, csy = 0, krx = 0, kry = 0, ntx = 0, nty = 0, segz = 0, nsegz = 0;
  int ax = 0, ay = 0, fx = 0, fy = 0;  // edge-flush tiling per axis (see Tb3dArgs)
};
Geom2D geom2d(int K, int nx, int ny, int seg);
// Geometry of a radius-R star pass: halo R*K per side (left halo rounded up to 4).
Geom2D geom_star(int R, int K, int nx, int ny, int seg);
// Geometry of a radius-R 3D star pass: 64 x 64 windows with a halo of R*K per side (csx = csy
// output cells per tile), streamed along z in segments of segz planes.
Geom3D geom_star3(int R, int K, int nx, int ny, int nz, int segz);
// Memory and arithmetic parts of a modelled time, summed over the passes (seconds).
struct ModelParts {
  double mem = 0.0, alu = 0.0;
};
Geom3D geom3d(int K, bool adj, int nx, int ny, int nz, int segz);
// Model time (seconds) of T steps with the given geometry.
double model_time_2d(const Geom2D& g, int nx, int ny, long T, bool hot, bool adj, bool phys = false,
                     ModelParts* parts = nullptr);
double model_time_3d(const Geom3D& g, int nx, int ny, int nz, long T, bool hot, bool adj, ModelParts* parts = nullptr);
double model_time_star(const Geom2D& g, int R, int nx, int ny, long T, ModelParts* parts = nullptr);
double model_time_star3(const Geom3D& g, int R, int nx, int ny, int nz, long T, ModelParts* parts = nullptr);
// The same for the balanced 3D launch of nwork workgroups (equal shares of column planes).
double model_time_3d_bal(const Geom3D& g, int nx, int ny, int nz, long T, bool hot, bool adj, int nwork,
                         ModelParts* parts = nullptr);
// Workgroups of a balanced 3D launch: `mult` per CU, fewer when the grid has too few column
// planes to give each at least a few times the pipeline depth.
int balanced_nwork3d(int K, bool adj, int nx, int ny, int nz, int mult);
// Choose segment lengths that balance the tile count against the device's concurrency.
int pick_seg2d(int K, int nx, int ny, int waves_per_cu);
int pick_segz3d(int K, bool adj, int nx, int ny, int nz, int wgs_per_cu);

DevCoef dev_coef(const stencil_coeffs_t& c, bool adjoint, bool phys = false);
bool coeffs_finite(const stencil_coeffs_t& c);

}  // namespace stn

struct stencil_plan_s {
  stencil_form_t form;
  int ndim, nx, ny, nz;
  int rad = 1;           // > 0 with star = true: a radius-rad star plan (stencil_create_star)
  bool star = false;
  StarCoef star_cf{};    // weights of the current stencil_run_star call (2D)
  Star3Coef star3_cf{};  // the same for a 3D plan
  const float* star_power = nullptr;  // power map of the current hotspot-form star run, or null
  size_t cells;
  hipStream_t stream;
  int device;
  stencil_tuning_t tuning;  // resolved
  int nwork3d = 0;          // 3D: > 0 selects the balanced launch with this many workgroups
  // blocking of the transposed (adjoint) passes: fused steps, segment length, balanced 3D
  // launch workgroups (0: tile launch)
  int adj_k = 0, adj_seg = 0, adj_nwork = 0;
  // 2D: edge tiles run on a second stream, concurrently with the interior tiles of a pass
  hipStream_t side = nullptr;
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;
  float* scratch = nullptr;
  // checkpoints of the last stencil_run_ckpt
  std::vector<float*> ckpts;
  int ckpt_every = 0;
  int ckpt_T = -1;
  // recompute verification
  float* verify_buf = nullptr;
  int* mismatch = nullptr;
};
