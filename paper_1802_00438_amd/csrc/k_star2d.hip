// Temporal-blocked radius-r 2D star-stencil kernels (diffusion form): instantiation table and
// the launch of one pass.  The kernels of radius 1-2 and 3-4 are compiled in two translation
// units of their own.
#include "star2d.hpp"

// Instantiated fused-step counts per radius: the level windows, K x (2R+1) rows of 4 cells,
// must fit the register file.
static const int kStarK1[] = {1, 2, 4, 8};
static const int kStarK2[] = {1, 2, 4, 5, 8};
static const int kStarK34[] = {1, 2, 4};

int star_instantiated(int R, const int** ks) {
  if (R == 1) { *ks = kStarK1; return 4; }
  if (R == 2) { *ks = kStarK2; return 5; }
  if (R == 3 || R == 4) { *ks = kStarK34; return 3; }
  *ks = nullptr;
  return 0;
}

hipError_t launch_star2d_r12(int R, int K, const Star2dArgs& a, hipStream_t s);
hipError_t launch_star2d_r34(int R, int K, const Star2dArgs& a, hipStream_t s);

hipError_t launch_star2d(int R, int K, const Star2dArgs& a, hipStream_t s) {
  if (R == 1 || R == 2) return launch_star2d_r12(R, K, a, s);
  if (R == 3 || R == 4) return launch_star2d_r34(R, K, a, s);
  return hipErrorInvalidValue;
}
