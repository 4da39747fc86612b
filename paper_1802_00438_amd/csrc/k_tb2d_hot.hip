// Temporal-blocked 2D hotspot kernels (forward).
#include "launch.hpp"
#define C(K) case K: if (full) TB_LAUNCH2D(K, true, false, false, true, a, s); else TB_LAUNCH2D(K, true, false, false, false, a, s);
hipError_t launch_tb2d_hot(int K, bool full, const Tb2dArgs& a, hipStream_t s) {
  switch (K) { C(4) C(8) C(12) C(16) default: return hipErrorInvalidValue; }
}
