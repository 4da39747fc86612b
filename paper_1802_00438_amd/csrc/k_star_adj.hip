// The transposed step of the radius-r star stencils (adjoint sweep of a star plan): the
// four-cells-per-lane kernel where rows are whole 16-byte groups, else one cell per thread.
#include "star_adjoint.hpp"

hipError_t launch_star_adjoint(const StarAdjArgs& a, hipStream_t s) {
  const long nb = star_adjoint_blocks(a);
  if (nb <= 0 || nb > 0x7fffffffL || a.rad < 1 || a.rad > kStarMaxR) return hipErrorInvalidValue;
  // four cells per lane where every row is whole 16-byte groups
  auto al16 = [](const void* p) { return (reinterpret_cast<uintptr_t>(p) & 15) == 0; };
  const bool v4 = (a.nx % 4) == 0 && al16(a.lam) && al16(a.out) && (!a.gp || al16(a.gp));
#define SA(D, R)                                                                                   \
  case R:                                                                                          \
    if (v4) hipLaunchKernelGGL((star_adjoint_v4_kernel<D, R>), dim3((unsigned)nb), dim3(64), 0, s, a); \
    else hipLaunchKernelGGL((star_adjoint_kernel<D, R>), dim3((unsigned)nb), dim3(256), 0, s, a);   \
    break;
  if (a.ndim == 3) {
    switch (a.rad) { SA(3, 1) SA(3, 2) SA(3, 3) SA(3, 4) default: return hipErrorInvalidValue; }
  } else {
    switch (a.rad) { SA(2, 1) SA(2, 2) SA(2, 3) SA(2, 4) default: return hipErrorInvalidValue; }
  }
#undef SA
  return hipGetLastError();
}
