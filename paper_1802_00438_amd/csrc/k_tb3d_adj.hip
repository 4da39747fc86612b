// Temporal-blocked 3D transposed-stencil (adjoint) kernels.
#include "launch.hpp"
#define C(K)                                                                                    \
  case K:                                                                                       \
    if (acc) {                                                                                  \
      if (full) TB_LAUNCH3D(K, kTb3dAdjR, kTb3dAdjNW, false, true, true, true, a, s);            \
      else TB_LAUNCH3D(K, kTb3dAdjR, kTb3dAdjNW, false, true, true, false, a, s);                \
    } else {                                                                                    \
      if (full) TB_LAUNCH3D(K, kTb3dAdjR, kTb3dAdjNW, false, true, false, true, a, s);           \
      else TB_LAUNCH3D(K, kTb3dAdjR, kTb3dAdjNW, false, true, false, false, a, s);               \
    }
hipError_t launch_tb3d_adj(int K, bool acc, bool full, const Tb3dArgs& a, hipStream_t s) {
  switch (K) { C(1) C(2) C(3) C(4) default: return hipErrorInvalidValue; }
}
