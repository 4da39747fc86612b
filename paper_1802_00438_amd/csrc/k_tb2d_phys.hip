// Temporal-blocked 2D kernels of the physical Hotspot 2D formula (Table 2 as printed).
#include "launch.hpp"
#define C(K) case K: if (full) TB_LAUNCH2D_F(K, true, false, false, true, true, a, s); else TB_LAUNCH2D_F(K, true, false, false, false, true, a, s);
hipError_t launch_tb2d_phys(int K, bool full, const Tb2dArgs& a, hipStream_t s) {
  switch (K) { C(4) C(8) C(12) C(16) default: return hipErrorInvalidValue; }
}

// Transposed step of the physical form (its linear part is symmetric), with or without grad_p.
#define CA(K)                                                                          \
  case K:                                                                              \
    if (acc) {                                                                         \
      if (full) TB_LAUNCH2D_F(K, false, true, true, true, true, a, s);                 \
      else TB_LAUNCH2D_F(K, false, true, true, false, true, a, s);                     \
    } else {                                                                           \
      if (full) TB_LAUNCH2D_F(K, false, true, false, true, true, a, s);                \
      else TB_LAUNCH2D_F(K, false, true, false, false, true, a, s);                    \
    }
hipError_t launch_tb2d_phys_adj(int K, bool acc, bool full, const Tb2dArgs& a, hipStream_t s) {
  switch (K) { CA(4) CA(8) CA(12) default: return hipErrorInvalidValue; }
}
