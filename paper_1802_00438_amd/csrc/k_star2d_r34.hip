// Radius-r 2D star-stencil kernels, radius 3 and 4.
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

hipError_t launch_star2d_r34(int R, int K, const Star2dArgs& a, hipStream_t s) {
  switch (R) {
    case 3: switch (K) { SL(3, 1) SL(3, 2) SL(3, 4) default: return hipErrorInvalidValue; } break;
    case 4: switch (K) { SL(4, 1) SL(4, 2) SL(4, 4) default: return hipErrorInvalidValue; } break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}
