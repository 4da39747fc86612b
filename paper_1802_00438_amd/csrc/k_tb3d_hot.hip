// Temporal-blocked 3D hotspot kernels (forward).
#include "launch.hpp"
#define C(K) case K: if (full) TB_LAUNCH3D(K, tb3d_rows(K, true), tb3d_waves(K, true), true, false, false, true, a, s); \
                     else TB_LAUNCH3D(K, tb3d_rows(K, true), tb3d_waves(K, true), true, false, false, false, a, s);
hipError_t launch_tb3d_hot(int K, bool full, const Tb3dArgs& a, hipStream_t s) {
  switch (K) { C(1) C(2) C(3) C(4) default: return hipErrorInvalidValue; }
}
