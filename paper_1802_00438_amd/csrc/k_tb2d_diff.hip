// Temporal-blocked 2D diffusion kernels (forward).
#include "launch.hpp"
#define C(K) case K: if (full) TB_LAUNCH2D(K, false, false, false, true, a, s); else TB_LAUNCH2D(K, false, false, false, false, a, s);
hipError_t launch_tb2d_diff(int K, bool full, const Tb2dArgs& a, hipStream_t s) {
  switch (K) { C(4) C(8) C(12) C(16) C(20) C(24) default: return hipErrorInvalidValue; }
}
