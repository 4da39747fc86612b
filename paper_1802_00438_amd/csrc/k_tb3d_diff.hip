// Temporal-blocked 3D diffusion kernels (forward).
#include "launch.hpp"
#define C(K) case K: if (full) TB_LAUNCH3D(K, tb3d_rows(K, false), tb3d_waves(K, false), false, false, false, true, a, s); \
                     else TB_LAUNCH3D(K, tb3d_rows(K, false), tb3d_waves(K, false), false, false, false, false, a, s);
hipError_t launch_tb3d_diff(int K, bool full, const Tb3dArgs& a, hipStream_t s) {
  switch (K) { C(1) C(2) C(3) C(4) C(5) C(6) default: return hipErrorInvalidValue; }
}
