// plain.hpp -- one time step per launch (no temporal blocking).
//
// This is the comparator behind the roofline of the paper's Section 6.4: without temporal
// blocking every step reads the grid (and the power map) from HBM and writes it back, so its
// ceiling is HBM bandwidth divided by the bytes per cell update of Table 2 (8 B diffusion,
// 12 B hotspot).
//
// One wave per workgroup; lane l owns four consecutive x cells (one 16-byte access) of a
// 256-column chunk and marches kPlainMR2 rows (2D) or a.mr3 planes (3D) along the slowest axis,
// keeping the previous, current and next row (plane) in registers and loading the one after
// next an iteration ahead, so every value along the marched axis is fetched once per step (plus
// two per strip).  The x neighbours beyond a lane's four cells come from the neighbouring lanes
// through DPP; only the first and last lane of a wave read theirs from memory.  In 3D the
// in-plane y neighbours are the rows that the waves of the adjacent rows stream, read at the
// current plane (by which time those waves have brought them into L2): workgroups are ordered
// chunk, then row, then strip, and mapped so that each XCD runs a contiguous range of them, so
// a row is fetched from HBM once and read by its neighbours from the XCD's L2.  (Streaming
// several rows per wave, with the neighbour rows loaded either with the plane ahead or at the
// current plane, measured 8-35% slower on the 512^3 grid.)
#pragma once
#include "device_common.hpp"

struct PlainArgs {
  const float* src;
  float* dst;
  const float* power;  // forward hotspot
  float* gp;           // adjoint hotspot accumulator (grad_p += cp * src), or null
  int nx, ny, nz, ndim;
  int chunks;          // 256-column chunks per row
  int vec;             // 1: nx % 4 == 0 and 16-byte aligned buffers
  int stream;          // 1: nontemporal stores of the output (grids far larger than the cache)
  int mr3;             // 3D: planes marched per wave (the strip length along z)
  DevCoef cf;
};

// Rows marched per wave in 2D (32 measured 3% slower).  In 3D the strip length is a launch
// argument (PlainArgs::mr3) that the host sizes to the grid.
constexpr int kPlainMR2 = 16;

// four consecutive cells starting at x0 of row r (clamped beyond nx on the scalar path)
__device__ __forceinline__ void plain_ld4(const float* r, int x0, int nx, bool vec, float (&o)[4]) {
  if (vec) {
    const float4 t = *reinterpret_cast<const float4*>(r + x0);
    o[0] = t.x; o[1] = t.y; o[2] = t.z; o[3] = t.w;
  } else {
#pragma unroll
    for (int v = 0; v < 4; ++v) o[v] = r[min(x0 + v, nx - 1)];
  }
}

// PHYS (2D only): Table 2's physical Hotspot 2D formula in its printed order (see DevCoef for
// where its parameters travel); with ADJ, its symmetric linear part (no power, TEMP_AMB = 0)
// as the transposed step.
template <bool HOT, bool ADJ, bool ACC, bool PHYS = false>
__global__ __launch_bounds__(64) void plain_kernel(PlainArgs a) {
  static_assert(!PHYS || (HOT && !ADJ && !ACC) || (!HOT && ADJ), "physical form: forward hotspot or transposed step");
  const int b = xcd_remap(blockIdx.x, gridDim.x);
  const int chunk = b % a.chunks;
  const int strip = b / a.chunks;  // y-strips (2D) or (row y, z-strip) pairs (3D)
  const int lane = threadIdx.x;
  const int x0 = chunk * 256 + lane * 4;
  if (x0 >= a.nx) return;
  const bool vec = a.vec != 0;
  const int cnt = min(4, a.nx - x0);
  const size_t plane = (size_t)a.ny * a.nx;
  // marched axis: y (2D) or z (3D); the fixed in-plane row of a 3D wave is y
  int y = 0, s0, ns;
  if (a.ndim == 2) {
    s0 = strip * kPlainMR2;
    ns = a.ny;
  } else {
    y = strip % a.ny;
    s0 = (strip / a.ny) * a.mr3;
    ns = a.nz;
  }
  const int s1 = min(s0 + (a.ndim == 2 ? kPlainMR2 : a.mr3), ns);
  const size_t stride = a.ndim == 2 ? (size_t)a.nx : plane;  // distance between marched rows
  const float* sbase = a.src + (a.ndim == 2 ? 0 : (size_t)y * a.nx);
  const int ym = y > 0 ? y - 1 : 0, yp = y < a.ny - 1 ? y + 1 : a.ny - 1;
  const bool top = (a.ndim == 3) && (y == 0), bot = (a.ndim == 3) && (y == a.ny - 1);
  float prv[4], cur[4], nxt[4], nn[4];
  plain_ld4(sbase + (size_t)max(s0 - 1, 0) * stride, x0, a.nx, vec, prv);
  plain_ld4(sbase + (size_t)s0 * stride, x0, a.nx, vec, cur);
  plain_ld4(sbase + (size_t)min(s0 + 1, ns - 1) * stride, x0, a.nx, vec, nxt);
  for (int s = s0; s < s1; ++s) {
    plain_ld4(sbase + (size_t)min(s + 2, ns - 1) * stride, x0, a.nx, vec, nn);  // one ahead
    const float* cr = sbase + (size_t)s * stride;
    // x neighbours: the neighbouring lanes' cells; a wave's first and last lane read theirs
    float left = from_lower(cur[3]);
    float right = from_upper(cur[0]);
    if (lane == 0) left = (x0 > 0) ? cr[x0 - 1] : cur[0];
    if (lane == 63 || x0 + 4 >= a.nx) {
      // the row's last cell when it falls inside this lane (a select chain, not an indexed
      // register array, which would live in scratch memory)
      const float last = cnt == 1 ? cur[0] : (cnt == 2 ? cur[1] : (cnt == 3 ? cur[2] : cur[3]));
      right = (x0 + 4 < a.nx) ? cr[x0 + 4] : last;
    }
    float yn[4], ys[4], p4[4], g4[4];
    if (a.ndim == 3) {
      const float* pl = a.src + (size_t)s * plane;
      plain_ld4(pl + (size_t)ym * a.nx, x0, a.nx, vec, yn);
      plain_ld4(pl + (size_t)yp * a.nx, x0, a.nx, vec, ys);
    }
    const size_t off = (size_t)s * stride + (a.ndim == 2 ? 0 : (size_t)y * a.nx);
    if constexpr (HOT && !ADJ) plain_ld4(a.power + off, x0, a.nx, vec, p4);
    if constexpr (ACC) plain_ld4(a.gp + off, x0, a.nx, vec, g4);
    const bool slo = (s == 0), shi = (s == ns - 1);  // marched-axis edges (uniform per row)
    float o[4];
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int x = x0 + v;
      const float c = cur[v];
      const bool l = (x == 0), rr = (x == a.nx - 1);
      const float xm = l ? c : ((v == 0) ? left : cur[v - 1]);
      const float xp = rr ? c : ((v == 3) ? right : cur[v + 1]);
      float wxm = a.cf.wx_m, wxp = a.cf.wx_p;
      if constexpr (ADJ) {
        if (l) wxm = a.cf.wx_p;
        if (rr) wxp = a.cf.wx_m;
      }
      float acc;
      float q = 0.0f;
      if constexpr (HOT && !ADJ && !PHYS) q = __builtin_fmaf(a.cf.cp, p4[v], a.cf.kamb);
      if constexpr (PHYS) {
        const float yn2 = slo ? c : prv[v], ys2 = shi ? c : nxt[v];
        const float dy = __builtin_fmaf(-2.0f, c, yn2 + ys2);  // (n + s) - 2c, one rounding each
        const float dx = __builtin_fmaf(-2.0f, c, xp + xm);    // (e + w) - 2c
        const float dz = a.cf.kamb - c;                        // TEMP_AMB - c
        acc = __builtin_fmaf(dy, a.cf.wy_m, (HOT && !ADJ) ? p4[v] : 0.0f);
        acc = __builtin_fmaf(dx, a.cf.wx_m, acc);
        acc = __builtin_fmaf(dz, a.cf.wz_m, acc);
        acc = __builtin_fmaf(a.cf.cp, acc, c);
      } else if (a.ndim == 2) {
        // marched axis is y: prv = row y-1, nxt = row y+1
        float cym = a.cf.wy_m, cyp = a.cf.wy_p;
        if constexpr (ADJ) {
          if (slo) cym = a.cf.wy_p;
          if (shi) cyp = a.cf.wy_m;
        }
        acc = upd2<HOT && !ADJ>(a.cf.c0, c, wxm, xm, wxp, xp, cyp, shi ? c : nxt[v], cym, slo ? c : prv[v], q);
      } else {
        float cym = a.cf.wy_m, cyp = a.cf.wy_p, czm = a.cf.wz_m, czp = a.cf.wz_p;
        if constexpr (ADJ) {
          if (top) cym = a.cf.wy_p;
          if (bot) cyp = a.cf.wy_m;
          if (slo) czm = a.cf.wz_p;
          if (shi) czp = a.cf.wz_m;
        }
        acc = upd2<HOT && !ADJ>(a.cf.c0, c, wxm, xm, wxp, xp, cyp, bot ? c : ys[v], cym, top ? c : yn[v], q);
        acc = __builtin_fmaf(czm, slo ? c : prv[v], acc);
        acc = __builtin_fmaf(czp, shi ? c : nxt[v], acc);
      }
      o[v] = acc;
      if constexpr (ACC) g4[v] = __builtin_fmaf(a.cf.cp, c, g4[v]);
    }
    float* dr = a.dst + off;
    if (vec) {
      store4(dr, x0, a.nx, o[0], o[1], o[2], o[3], a.stream != 0);
      if constexpr (ACC) *reinterpret_cast<float4*>(a.gp + off + x0) = make_float4(g4[0], g4[1], g4[2], g4[3]);
    } else {
#pragma unroll
      for (int v = 0; v < 4; ++v)
        if (v < cnt) {
          dr[x0 + v] = o[v];
          if constexpr (ACC) a.gp[off + x0 + v] = g4[v];
        }
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      prv[v] = cur[v];
      cur[v] = nxt[v];
      nxt[v] = nn[v];
    }
  }
}

// Workgroups of one plain launch: (256-column chunks) x (strips along the marched axis).
inline int plain_blocks(const PlainArgs& a) {
  if (a.ndim == 2) return a.chunks * ((a.ny + kPlainMR2 - 1) / kPlainMR2);
  return a.chunks * a.ny * ((a.nz + a.mr3 - 1) / a.mr3);
}
