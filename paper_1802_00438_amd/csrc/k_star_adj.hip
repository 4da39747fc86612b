// The transposed step of the radius-r star stencils (adjoint sweep of a star plan).
#include "star_adjoint.hpp"

hipError_t launch_star_adjoint(const StarAdjArgs& a, hipStream_t s) {
  const long nb = star_adjoint_blocks(a);
  if (nb <= 0 || nb > 0x7fffffffL || a.rad < 1 || a.rad > kStarMaxR) return hipErrorInvalidValue;
#define SA(D, R)                                                                                   \
  case R:                                                                                          \
    hipLaunchKernelGGL((star_adjoint_kernel<D, R>), dim3((unsigned)nb), dim3(256), 0, s, a);        \
    break;
  if (a.ndim == 3) {
    switch (a.rad) { SA(3, 1) SA(3, 2) SA(3, 3) SA(3, 4) default: return hipErrorInvalidValue; }
  } else {
    switch (a.rad) { SA(2, 1) SA(2, 2) SA(2, 3) SA(2, 4) default: return hipErrorInvalidValue; }
  }
#undef SA
  return hipGetLastError();
}
