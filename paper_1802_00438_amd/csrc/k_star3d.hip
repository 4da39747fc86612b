// Temporal-blocked radius-r 3D star-stencil kernels (diffusion form): instantiation table and
// the launch of one pass.
#include "star3d.hpp"

// Instantiated fused-step counts per radius: the K levels' held planes and partial sums (2R+1
// values per lane cell and level) must fit 128 VGPRs (16 waves per workgroup) without spills.
// Every count from 1 to the largest is instantiated: a pass runs on the kernel whose K is the
// number of steps it fuses.
static const int kStar3K1[] = {1, 2, 3};
static const int kStar3K23[] = {1, 2};
static const int kStar3K4[] = {1};

int star3_instantiated(int R, const int** ks) {
  if (R == 1) { *ks = kStar3K1; return 3; }
  if (R == 2 || R == 3) { *ks = kStar3K23; return 2; }
  if (R == 4) { *ks = kStar3K4; return 1; }
  *ks = nullptr;
  return 0;
}

#define S3(R, K)                                                                                        \
  case K:                                                                                               \
    if (a.power) hipLaunchKernelGGL((star3d_kernel<R, K, true>), dim3(nb), dim3(kStar3Threads), 0, s, a); \
    else hipLaunchKernelGGL((star3d_kernel<R, K, false>), dim3(nb), dim3(kStar3Threads), 0, s, a);       \
    break;

hipError_t launch_star3d(int R, int K, const Star3dArgs& a, hipStream_t s) {
  const long nbl = (long)a.ntx * a.nty * a.nsegz;
  if (nbl <= 0 || nbl > 0x7fffffffL || a.keff != K || a.cs != kStar3W - 2 * R * K)
    return hipErrorInvalidValue;
  const unsigned nb = (unsigned)nbl;
  switch (R) {
    case 1: switch (K) { S3(1, 1) S3(1, 2) S3(1, 3) default: return hipErrorInvalidValue; } break;
    case 2: switch (K) { S3(2, 1) S3(2, 2) default: return hipErrorInvalidValue; } break;
    case 3: switch (K) { S3(3, 1) S3(3, 2) default: return hipErrorInvalidValue; } break;
    case 4: switch (K) { S3(4, 1) default: return hipErrorInvalidValue; } break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}
