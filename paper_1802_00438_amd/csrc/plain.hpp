// plain.hpp -- one time step per launch (no temporal blocking).
//
// This is the comparator of the paper's Section 6.4 roofline ("full utilization of external
// memory bandwidth ... without temporal blocking"): every step reads the grid (and the power
// map) from HBM and writes it back, so its ceiling is HBM bandwidth / bytes per cell update
// (Table 2: 8 B diffusion, 12 B hotspot).  Each thread updates four consecutive x cells of
// one row with 16-byte accesses; the y/z neighbour rows are re-read through L2.
#pragma once
#include "device_common.hpp"

struct PlainArgs {
  const float* src;
  float* dst;
  const float* power;  // forward hotspot
  float* gp;           // adjoint hotspot accumulator (grad_p += cp * src), or null
  int nx, ny, nz, ndim;
  int chunks;          // 1024-column chunks per row
  int vec;             // 1: nx % 4 == 0 and 16-byte aligned buffers
  DevCoef cf;
};

template <bool HOT, bool ADJ, bool ACC>
__global__ __launch_bounds__(256) void plain_kernel(PlainArgs a) {
  const int chunk = blockIdx.x % a.chunks;
  const int row = blockIdx.x / a.chunks;  // row index over (z, y)
  const int y = row % a.ny;
  const int z = row / a.ny;
  const int x0 = chunk * 1024 + threadIdx.x * 4;
  if (x0 >= a.nx) return;
  const size_t plane = (size_t)a.ny * a.nx;
  const size_t off = (size_t)z * plane + (size_t)y * a.nx;
  const float* cr = a.src + off;
  const int ym = y > 0 ? y - 1 : 0, yp = y < a.ny - 1 ? y + 1 : a.ny - 1;
  const float* nr = a.src + (size_t)z * plane + (size_t)ym * a.nx;
  const float* sr = a.src + (size_t)z * plane + (size_t)yp * a.nx;
  const int zm = z > 0 ? z - 1 : 0, zp = z < a.nz - 1 ? z + 1 : a.nz - 1;
  const float* br = a.src + (size_t)zm * plane + (size_t)y * a.nx;
  const float* ar = a.src + (size_t)zp * plane + (size_t)y * a.nx;
  const bool top = (y == 0), bot = (y == a.ny - 1);
  const bool zlo = (z == 0), zhi = (z == a.nz - 1);
  float cym = a.cf.wy_m, cyp = a.cf.wy_p, czm = a.cf.wz_m, czp = a.cf.wz_p;
  if constexpr (ADJ) {
    if (top) cym = a.cf.wy_p;
    if (bot) cyp = a.cf.wy_m;
    if (zlo) czm = a.cf.wz_p;
    if (zhi) czp = a.cf.wz_m;
  }
  // 16-byte vector path for whole, aligned 4-cell groups; scalar path for ragged rows
  float c[4], n4[4], s4[4], b4[4], a4[4], p4[4], g4[4];
  const bool vec = a.vec != 0;
  const int cnt = min(4, a.nx - x0);
  if (vec) {
    const float4 tc = *reinterpret_cast<const float4*>(cr + x0);
    const float4 tn = *reinterpret_cast<const float4*>(nr + x0);
    const float4 ts = *reinterpret_cast<const float4*>(sr + x0);
    c[0] = tc.x; c[1] = tc.y; c[2] = tc.z; c[3] = tc.w;
    n4[0] = tn.x; n4[1] = tn.y; n4[2] = tn.z; n4[3] = tn.w;
    s4[0] = ts.x; s4[1] = ts.y; s4[2] = ts.z; s4[3] = ts.w;
    if (a.ndim == 3) {
      const float4 tb = *reinterpret_cast<const float4*>(br + x0);
      const float4 ta = *reinterpret_cast<const float4*>(ar + x0);
      b4[0] = tb.x; b4[1] = tb.y; b4[2] = tb.z; b4[3] = tb.w;
      a4[0] = ta.x; a4[1] = ta.y; a4[2] = ta.z; a4[3] = ta.w;
    }
    if constexpr (HOT && !ADJ) {
      const float4 tp = *reinterpret_cast<const float4*>(a.power + off + x0);
      p4[0] = tp.x; p4[1] = tp.y; p4[2] = tp.z; p4[3] = tp.w;
    }
    if constexpr (ACC) {
      const float4 tg = *reinterpret_cast<const float4*>(a.gp + off + x0);
      g4[0] = tg.x; g4[1] = tg.y; g4[2] = tg.z; g4[3] = tg.w;
    }
  } else {
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int x = min(x0 + v, a.nx - 1);
      c[v] = cr[x]; n4[v] = nr[x]; s4[v] = sr[x];
      if (a.ndim == 3) { b4[v] = br[x]; a4[v] = ar[x]; }
      if constexpr (HOT && !ADJ) p4[v] = a.power[off + x];
      if constexpr (ACC) g4[v] = a.gp[off + x];
    }
  }
  const float left = (x0 > 0) ? cr[x0 - 1] : c[0];
  const float right = (x0 + 4 < a.nx) ? cr[x0 + 4] : c[cnt - 1];
  float o[4];
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int x = x0 + v;
    const bool l = (x == 0), rr = (x == a.nx - 1);
    const float xm = (v == 0) ? left : c[v - 1];
    const float xp = rr ? c[v] : ((v == 3) ? right : c[v + 1]);
    float wxm = a.cf.wx_m, wxp = a.cf.wx_p;
    if constexpr (ADJ) {
      if (l) wxm = a.cf.wx_p;
      if (rr) wxp = a.cf.wx_m;
    }
    const float yv_m = top ? c[v] : n4[v];
    const float yv_p = bot ? c[v] : s4[v];
    float acc = upd2(a.cf.c0, c[v], wxm, l ? c[v] : xm, wxp, xp, cyp, yv_p, cym, yv_m);
    if (a.ndim == 3) {
      acc = __builtin_fmaf(czm, zlo ? c[v] : b4[v], acc);
      acc = __builtin_fmaf(czp, zhi ? c[v] : a4[v], acc);
    }
    if constexpr (HOT && !ADJ) acc = acc + __builtin_fmaf(a.cf.cp, p4[v], a.cf.kamb);
    o[v] = acc;
    if constexpr (ACC) g4[v] = __builtin_fmaf(a.cf.cp, c[v], g4[v]);
  }
  if (vec) {
    *reinterpret_cast<float4*>(a.dst + off + x0) = make_float4(o[0], o[1], o[2], o[3]);
    if constexpr (ACC) *reinterpret_cast<float4*>(a.gp + off + x0) = make_float4(g4[0], g4[1], g4[2], g4[3]);
  } else {
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      if (v < cnt) {
        a.dst[off + x0 + v] = o[v];
        if constexpr (ACC) a.gp[off + x0 + v] = g4[v];
      }
    }
  }
}

