// Temporal-blocked radius-r 2D star-stencil kernels (diffusion form).
#include "star2d.hpp"

// Instantiated fused-step counts per radius: the level windows, K x (2R+1) rows of 4 cells,
// must fit the register file.
static const int kStarK1[] = {1, 2, 4, 8};
static const int kStarK2[] = {1, 2, 4, 8};
static const int kStarK3[] = {1, 2, 4};
static const int kStarK4[] = {1, 2, 4};

int star_instantiated(int R, const int** ks) {
  switch (R) {
    case 1: *ks = kStarK1; return 4;
    case 2: *ks = kStarK2; return 4;
    case 3: *ks = kStarK3; return 3;
    case 4: *ks = kStarK4; return 3;
  }
  *ks = nullptr;
  return 0;
}

inline int star2d_tiles(const Star2dArgs& a) { return a.ntx * a.nseg; }

#define SL(R, K) case K: hipLaunchKernelGGL((star2d_kernel<R, K>), dim3(star2d_tiles(a)), dim3(64), 0, s, a); break;
hipError_t launch_star2d(int R, int K, const Star2dArgs& a, hipStream_t s) {
  switch (R) {
    case 1: switch (K) { SL(1, 1) SL(1, 2) SL(1, 4) SL(1, 8) default: return hipErrorInvalidValue; } break;
    case 2: switch (K) { SL(2, 1) SL(2, 2) SL(2, 4) SL(2, 8) default: return hipErrorInvalidValue; } break;
    case 3: switch (K) { SL(3, 1) SL(3, 2) SL(3, 4) default: return hipErrorInvalidValue; } break;
    case 4: switch (K) { SL(4, 1) SL(4, 2) SL(4, 4) default: return hipErrorInvalidValue; } break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}
