// Temporal-blocked 2D transposed-stencil (adjoint) kernels.
#include "launch.hpp"
#define C(K)                                                                          \
  case K:                                                                             \
    if (acc) {                                                                        \
      if (full) TB_LAUNCH2D(K, false, true, true, true, a, s);                        \
      else TB_LAUNCH2D(K, false, true, true, false, a, s);                            \
    } else {                                                                          \
      if (full) TB_LAUNCH2D(K, false, true, false, true, a, s);                       \
      else TB_LAUNCH2D(K, false, true, false, false, a, s);                           \
    }
hipError_t launch_tb2d_adj(int K, bool acc, bool full, const Tb2dArgs& a, hipStream_t s) {
  switch (K) { C(4) C(8) C(12) default: return hipErrorInvalidValue; }
}
