// device_common.hpp -- small device helpers shared by the gfx950 stencil kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

// Weights as seen by a kernel.  The names give the *position* of the value each weight
// multiplies (x-1, x+1, y-1, y+1, z-1, z+1), not a direction of flow:
//   forward step (Table 2):   wx_m = cw, wx_p = ce, wy_m = cn, wy_p = cs, wz_m = cb, wz_p = ca
//   transposed step (adjoint): wx_m = ce, wx_p = cw, wy_m = cs, wy_p = cn, wz_m = ca, wz_p = cb
// kamb = c_amb * t_amb rounded once in FP32; cp multiplies the power map.
// Physical Hotspot 2D (Table 2 as printed): wx_m = wx_p = Rx_1, wy_m = wy_p = Ry_1,
// wz_m = Rz_1, cp = sdc, kamb = TEMP_AMB; c0 and wz_p are unused.
struct DevCoef {
  float c0, wx_m, wx_p, wy_m, wy_p, wz_m, wz_p, cp, kamb;
};

// The canonical evaluation order of one cell update: centre, x-1, x+1, y+1, y-1, z-1, z+1
// (the term order of Table 2), every step an FP32 fused multiply-add.  The hotspot source q
// (time-invariant) starts the sum: acc = fma(c0, c, q); diffusion starts from c0 * c.
template <bool SRC>
__device__ __forceinline__ float centre_term(float c0, float c, float q) {
  if constexpr (SRC) return __builtin_fmaf(c0, c, q);
  else return c0 * c;
}

template <bool SRC = false>
__device__ __forceinline__ float upd2(float c0, float c, float wxm, float xm, float wxp, float xp,
                                      float wyp, float yp, float wym, float ym, float q = 0.0f) {
  float acc = centre_term<SRC>(c0, c, q);
  acc = __builtin_fmaf(wxm, xm, acc);
  acc = __builtin_fmaf(wxp, xp, acc);
  acc = __builtin_fmaf(wyp, yp, acc);
  acc = __builtin_fmaf(wym, ym, acc);
  return acc;
}

// Vector store of 4 consecutive floats at element x of a row that starts at `row`, a
// wave-uniform, 16-byte aligned address of a row of n floats (n < 2^29); x is the lane's own.
// With stream set (a wave-uniform launch argument) the store carries the nontemporal hint, so
// the written lines are not kept in the caches.  That pays on grids far larger than the chip's
// 256 MB last-level cache, where an output line is never read back before it would be evicted
// and keeping it only evicts input rows that neighbouring tiles still read; on grids that fit,
// the next pass reads its input back from that cache, and the hint costs.  The streaming store
// is a raw buffer store over the row, whose cache policy is an immediate operand: two pointer
// stores that differ only in the hint are folded into one by the compiler, which drops the
// hint.
typedef float f32x4_t __attribute__((ext_vector_type(4)));
typedef unsigned u32x4_t __attribute__((ext_vector_type(4)));
constexpr int kRawBufWord3 = 0x00020000;  // descriptor word 3: raw buffer, 32-bit data format
constexpr int kCachePolicyNT = 2;         // cache-policy immediate of a buffer access: nt

__device__ __forceinline__ void store4(float* row, int x, int n, float a, float b, float c, float d, bool stream) {
  const f32x4_t v = {a, b, c, d};
  if (stream) {
    const __amdgpu_buffer_rsrc_t r = __builtin_amdgcn_make_buffer_rsrc(row, 0, n * 4, kRawBufWord3);
    __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(u32x4_t, v), r, x * 4, 0, kCachePolicyNT);
  } else {
    *reinterpret_cast<f32x4_t*>(row + x) = v;
  }
}

// Cross-lane moves inside one 64-wide wavefront through DPP (no LDS traffic):
// from_lower(x) returns lane i-1's x on lane i, from_upper(x) lane i+1's x.  The end lanes
// receive 0; they only ever hold halo columns whose values are never stored.
__device__ __forceinline__ float from_lower(float x) {
  return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, x),
                                                               0x138 /* wave_shr:1 */, 0xf, 0xf, true));
}
__device__ __forceinline__ float from_upper(float x) {
  return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, x),
                                                               0x130 /* wave_shl:1 */, 0xf, 0xf, true));
}

// The same moves where the end lane keeps `own` (bound_ctrl off: an invalid source lane leaves
// the destination at its old value).  In a window flush with the grid edge, lane 0 holds x = 0
// and lane 63 holds x = nx-1, so they receive their own value: the clamp-to-edge neighbour.
__device__ __forceinline__ float from_lower_or(float x, float own) {
  return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(__builtin_bit_cast(int, own), __builtin_bit_cast(int, x),
                                                               0x138 /* wave_shr:1 */, 0xf, 0xf, false));
}
__device__ __forceinline__ float from_upper_or(float x, float own) {
  return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(__builtin_bit_cast(int, own), __builtin_bit_cast(int, x),
                                                               0x130 /* wave_shl:1 */, 0xf, 0xf, false));
}

// The x-1 and x+1 terms of an interior row fused with their cross-lane moves: al += wl * xl of
// lane i-1 and au += wu * xu of lane i+1, each one v_fmac_f32 whose first source is read
// through DPP -- the same single-rounding FMA as fma(wl, from_lower(xl), al).  The compiler
// does not form these itself because a DPP instruction cannot take its other operand from an
// SGPR, so the weights are passed in VGPRs.  One "s_nop 1" before the pair provides the two
// wait states a DPP read needs after a VALU write of its source register.  End lanes read 0
// and leave their accumulator unchanged; they only ever hold halo columns.
__device__ __forceinline__ void fma_pair_dpp(float wl, float xl, float& al, float wu, float xu, float& au) {
  asm("s_nop 1\n\tv_fmac_f32_dpp %0, %2, %3 wave_shr:1 row_mask:0xf bank_mask:0xf bound_ctrl:1\n\t"
      "v_fmac_f32_dpp %1, %4, %5 wave_shl:1 row_mask:0xf bank_mask:0xf bound_ctrl:1"
      : "+v"(al), "+v"(au)
      : "v"(xl), "v"(wl), "v"(xu), "v"(wu));
}

// Single fused forms: acc += w * (x of lane i-1), acc += w * (x of lane i+1), each one
// v_fmac_f32_dpp behind its own "s_nop 1" (the DPP read hazard); end lanes add w * 0.
__device__ __forceinline__ float fma_from_lower_dpp(float w, float x, float acc) {
  asm("s_nop 1\n\tv_fmac_f32_dpp %0, %1, %2 wave_shr:1 row_mask:0xf bank_mask:0xf bound_ctrl:1"
      : "+v"(acc)
      : "v"(x), "v"(w));
  return acc;
}
__device__ __forceinline__ float fma_from_upper_dpp(float w, float x, float acc) {
  asm("s_nop 1\n\tv_fmac_f32_dpp %0, %1, %2 wave_shl:1 row_mask:0xf bank_mask:0xf bound_ctrl:1"
      : "+v"(acc)
      : "v"(x), "v"(w));
  return acc;
}

// The same pairing for sums: sl = (xl of lane i-1) + yl and su = (xu of lane i+1) + yu, each
// one v_add_f32 whose first source is read through DPP (end lanes read 0; halo columns only).
// The outputs are early-clobber: the first add must not overwrite an operand of the second.
__device__ __forceinline__ void add_pair_dpp(float xl, float yl, float& sl, float xu, float yu, float& su) {
  asm("s_nop 1\n\tv_add_f32_dpp %0, %2, %3 wave_shr:1 row_mask:0xf bank_mask:0xf bound_ctrl:1\n\t"
      "v_add_f32_dpp %1, %4, %5 wave_shl:1 row_mask:0xf bank_mask:0xf bound_ctrl:1"
      : "=&v"(sl), "=&v"(su)
      : "v"(xl), "v"(yl), "v"(xu), "v"(yu));
}

// gfx950 dispatches consecutive workgroup ids round-robin over its 8 XCDs, each with a
// private L2.  Remap so that each XCD receives a contiguous run of logical tile ids (and
// so shares the overlapping halo reads of neighbouring tiles in its own L2).  Bijective
// on [0, n): the tail that does not fill all 8 XCDs evenly keeps its id.
__device__ __forceinline__ int xcd_remap(int b, int n) {
  const int q = n >> 3;
  if (b < (q << 3)) return (b & 7) * q + (b >> 3);
  return b;
}

__device__ __forceinline__ int clampi(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }

// Agent-scope acquire/release helpers for cross-workgroup flags (persistent kernels).
__device__ __forceinline__ int ld_acquire(const int* p) {
  return __hip_atomic_load(p, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_release(int* p, int v) {
  __hip_atomic_store(p, v, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
}
