// Radius-r 2D star-stencil kernels, radius 1 and 2.
#include "star2d.hpp"

#define SL(R, K)                                                                                                \
  case K:                                                                                                       \
    if (a.power) {                                                                                              \
      if (a.keff == K) hipLaunchKernelGGL((star2d_kernel<R, K, true, true>), dim3(a.ntx * a.nseg), dim3(64), 0, s, a); \
      else hipLaunchKernelGGL((star2d_kernel<R, K, false, true>), dim3(a.ntx * a.nseg), dim3(64), 0, s, a);    \
    } else {                                                                                                    \
      if (a.keff == K) hipLaunchKernelGGL((star2d_kernel<R, K, true, false>), dim3(a.ntx * a.nseg), dim3(64), 0, s, a); \
      else hipLaunchKernelGGL((star2d_kernel<R, K, false, false>), dim3(a.ntx * a.nseg), dim3(64), 0, s, a);   \
    }                                                                                                           \
    break;

hipError_t launch_star2d_r12(int R, int K, const Star2dArgs& a, hipStream_t s) {
  switch (R) {
    case 1: switch (K) { SL(1, 1) SL(1, 2) SL(1, 4) SL(1, 8) default: return hipErrorInvalidValue; } break;
    case 2: switch (K) { SL(2, 1) SL(2, 2) SL(2, 4) SL(2, 5) SL(2, 8) default: return hipErrorInvalidValue; } break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}
