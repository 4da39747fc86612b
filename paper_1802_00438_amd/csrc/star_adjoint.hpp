// star_adjoint.hpp -- one transposed step of a radius-r star stencil (the adjoint sweep of a
// star plan), one launch per step.
//
// Method: the forward step (paper Eq. 1 and Eq. 2 with a general radius; Section 5.1's clamp at
// every distance) reads, for cell i and each directional weight, the neighbour at
// clamp(i + offset).  Its transpose gives cell j the weight of every (cell i, term) whose
// clamped neighbour is j.  Along one axis of length n, for the weight of the minus direction
// (x-d: w_d, y-d: n_d, z-d: b_d) and of the plus direction (x+d: e_d, y+d: s_d, z+d: a_d):
//   * minus weight: from cell j+d if it is inside the grid (zero outside); at j = 0 from every
//     cell 0..min(d, n-1), whose minus neighbour clamps to 0;
//   * plus weight: from cell j-d if it is inside the grid; at j = n-1 from every cell
//     max(n-1-d, 0)..n-1, whose plus neighbour clamps to n-1;
// and the centre weight from cell j itself.  The source term of the hotspot form does not
// depend on the state, so both forms share this step; the hotspot form also accumulates
// grad_p += cp * lambda (the step's input) at every step.
//
// gfx950 mapping: a thread owns one x cell and marches it along the slowest axis (y in 2D, z
// in 3D) over kAdjMS cells, keeping the 2R+1 values of that axis around the current cell in
// registers (zero beyond the grid, so the edge sums above are plain sums over the window); the
// in-plane neighbours are loaded, and workgroups (256 consecutive x cells) are ordered x, then
// y, then strip and mapped so that each XCD runs a contiguous range of them, so those loads
// hit L1/L2.  HBM then sees about one read and one write of lambda per step (plus grad_p's
// read and write in the hotspot form): 8 B (16 B) per cell and step, the plain kernel's
// roofline.
#pragma once
#include "device_common.hpp"
#include "star2d.hpp"

struct StarAdjArgs {
  const float* lam;  // lambda_t
  float* out;        // lambda_{t-1}
  float* gp;         // hotspot form: grad_p, accumulated; else null
  int nx, ny, nz, ndim, rad;
  int nbx;           // workgroups per row of x
  int stream;        // 1: nontemporal stores of lambda_{t-1} (grids far larger than the cache)
  float c0, cp;
  float wm[3][kStarMaxR], wp[3][kStarMaxR];  // per axis (x, y, z): minus and plus weights by distance
};

constexpr int kAdjMS = 16;  // cells marched per thread along the slowest axis

// The transposed terms of one in-plane axis for the cell at position j of n; p points at
// position 0 of that axis (the cell's other coordinates fixed), st is the axis stride.
template <int R>
__device__ __forceinline__ float adj_axis(float acc, int j, int n, const float* wm, const float* wp, const float* p,
                                          size_t st) {
#pragma unroll
  for (int d = 1; d <= R; ++d) {
    float vm, vp;
    if (j == 0) {
      vm = 0.0f;
      const int hi = min(d, n - 1);
      for (int i = 0; i <= hi; ++i) vm += p[i * st];
    } else {
      vm = (j + d <= n - 1) ? p[(j + d) * st] : 0.0f;
    }
    if (j == n - 1) {
      vp = 0.0f;
      for (int i = max(n - 1 - d, 0); i <= n - 1; ++i) vp += p[i * st];
    } else {
      vp = (j - d >= 0) ? p[(j - d) * st] : 0.0f;
    }
    acc = __builtin_fmaf(wm[d - 1], vm, acc);
    acc = __builtin_fmaf(wp[d - 1], vp, acc);
  }
  return acc;
}

template <int NDIM, int R>
__global__ __launch_bounds__(256) void star_adjoint_kernel(StarAdjArgs a) {
  const int b = xcd_remap(blockIdx.x, gridDim.x);
  const int bx = b % a.nbx;
  const int rest = b / a.nbx;
  const int x = bx * 256 + threadIdx.x;
  if (x >= a.nx) return;
  const size_t plane = (size_t)a.nx * a.ny;
  int y = 0, s0, ns;
  if constexpr (NDIM == 3) {
    y = rest % a.ny;
    s0 = (rest / a.ny) * kAdjMS;
    ns = a.nz;
  } else {
    s0 = rest * kAdjMS;
    ns = a.ny;
  }
  const int s1 = min(s0 + kAdjMS, ns);
  const size_t st = NDIM == 3 ? plane : (size_t)a.nx;            // stride of the marched axis
  const size_t col = NDIM == 3 ? (size_t)y * a.nx + x : (size_t)x;  // the thread's column
  const float* base = a.lam + col;
  const int ma = NDIM - 1;  // weights of the marched axis
  // win[k]: lambda at marched index s - R + k (zero beyond the grid)
  float win[2 * R + 1];
#pragma unroll
  for (int k = 0; k < 2 * R + 1; ++k) {
    const int i = s0 - R + k;
    win[k] = (i >= 0 && i < ns) ? base[(size_t)i * st] : 0.0f;
  }
  for (int s = s0; s < s1; ++s) {
    const int inext = s + R + 1;
    const float nextv = inext < ns ? base[(size_t)inext * st] : 0.0f;  // one ahead
    const float c = win[R];
    const size_t cell = (size_t)s * st + col;
    float acc = a.c0 * c;
    const float* rowp = a.lam + (size_t)s * st + (NDIM == 3 ? (size_t)y * a.nx : 0);
    acc = adj_axis<R>(acc, x, a.nx, a.wm[0], a.wp[0], rowp, 1);
    if constexpr (NDIM == 3) acc = adj_axis<R>(acc, y, a.ny, a.wm[1], a.wp[1], a.lam + (size_t)s * plane + x, a.nx);
#pragma unroll
    for (int d = 1; d <= R; ++d) {
      float vm = win[R + d], vp = win[R - d];
      if (s == 0) {  // every cell 0..d of the axis clamps its minus neighbour onto cell 0
        vm = 0.0f;
#pragma unroll
        for (int k = R; k <= R + d; ++k) vm += win[k];
      }
      if (s == ns - 1) {  // every cell ns-1-d..ns-1 clamps its plus neighbour onto cell ns-1
        vp = 0.0f;
#pragma unroll
        for (int k = R - d; k <= R; ++k) vp += win[k];
      }
      acc = __builtin_fmaf(a.wm[ma][d - 1], vm, acc);
      acc = __builtin_fmaf(a.wp[ma][d - 1], vp, acc);
    }
    a.out[cell] = acc;
    if (a.gp) a.gp[cell] = __builtin_fmaf(a.cp, c, a.gp[cell]);
#pragma unroll
    for (int k = 0; k < 2 * R; ++k) win[k] = win[k + 1];
    win[2 * R] = nextv;
  }
}

// The same step with four consecutive x cells per lane (one 16-byte access per row) and one
// wave per workgroup, for rows whose length is a multiple of 4 and 16-byte aligned buffers.
// The x neighbours up to distance 4 are in the lane or its neighbour lanes (DPP); the first
// and last lane of a wave load theirs.  A neighbour beyond the row is masked to zero, and the
// boundary sums of the row's first and last cell are sums over those same values.
template <int NDIM, int R>
__global__ __launch_bounds__(64) void star_adjoint_v4_kernel(StarAdjArgs a) {
  const int b = xcd_remap(blockIdx.x, gridDim.x);
  const int chunk = b % a.nbx;
  const int rest = b / a.nbx;
  const int lane = threadIdx.x;
  const int x0 = chunk * 256 + lane * 4;
  if (x0 >= a.nx) return;
  const size_t plane = (size_t)a.nx * a.ny;
  int y = 0, s0, ns;
  if constexpr (NDIM == 3) {
    y = rest % a.ny;
    s0 = (rest / a.ny) * kAdjMS;
    ns = a.nz;
  } else {
    s0 = rest * kAdjMS;
    ns = a.ny;
  }
  const int s1 = min(s0 + kAdjMS, ns);
  const size_t st = NDIM == 3 ? plane : (size_t)a.nx;
  const size_t roff = NDIM == 3 ? (size_t)y * a.nx : 0;  // the row's offset within a marched slice
  const float* base = a.lam + roff + x0;
  const int ma = NDIM - 1;
  auto ld4 = [](const float* p, float (&o)[4]) {
    const float4 t = *reinterpret_cast<const float4*>(p);
    o[0] = t.x; o[1] = t.y; o[2] = t.z; o[3] = t.w;
  };
  float win[2 * R + 1][4];
#pragma unroll
  for (int k = 0; k < 2 * R + 1; ++k) {
    const int i = s0 - R + k;
    if (i >= 0 && i < ns) {
      ld4(base + (size_t)i * st, win[k]);
    } else {
#pragma unroll
      for (int v = 0; v < 4; ++v) win[k][v] = 0.0f;
    }
  }
  const bool left = (x0 == 0), right = (x0 + 3 == a.nx - 1);
  for (int s = s0; s < s1; ++s) {
    float nxt[4] = {0.0f, 0.0f, 0.0f, 0.0f};
    if (s + R + 1 < ns) ld4(base + (size_t)(s + R + 1) * st, nxt);  // one ahead
    const float* rowp = a.lam + (size_t)s * st + roff;               // x = 0 of the cell's row
    // the cells x0-4 .. x0-1 (lo) and x0+4 .. x0+7 (up): neighbour lanes through DPP, the
    // wave's end lanes from memory; beyond the row they are masked below
    float lo[4], up[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      lo[k] = from_lower(win[R][k]);
      up[k] = from_upper(win[R][k]);
    }
    if (lane == 0 && x0 >= 4) ld4(rowp + x0 - 4, lo);
    if (lane == 63 && x0 + 4 < a.nx) ld4(rowp + x0 + 4, up);
    // value of the cell at offset o from x0 (o in -4..7), zero beyond the row
    auto X = [&](int o) -> float {
      const float v = o < 0 ? lo[(o + 4) & 3] : (o < 4 ? win[R][o & 3] : up[(o - 4) & 3]);
      return (x0 + o >= 0 && x0 + o <= a.nx - 1) ? v : 0.0f;
    };
    float acc[4];
#pragma unroll
    for (int v = 0; v < 4; ++v) acc[v] = a.c0 * win[R][v];
#pragma unroll
    for (int d = 1; d <= R; ++d) {
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        float vm = X(v + d), vp = X(v - d);
        if (v == 0 && left) {  // cells 0..d all clamp their x-d neighbour onto cell 0
          vm = 0.0f;
#pragma unroll
          for (int i = 0; i <= d; ++i) vm += X(i);
        }
        if (v == 3 && right) {  // cells nx-1-d..nx-1 all clamp their x+d neighbour onto nx-1
          vp = 0.0f;
#pragma unroll
          for (int i = 3 - d; i <= 3; ++i) vp += X(i);
        }
        acc[v] = __builtin_fmaf(a.wm[0][d - 1], vm, acc[v]);
        acc[v] = __builtin_fmaf(a.wp[0][d - 1], vp, acc[v]);
      }
    }
    if constexpr (NDIM == 3) {
      // y: the rows y +- d of plane s, zero beyond the grid; the first and last row gather the
      // clamped terms of every row within the distance
      const float* pl = a.lam + (size_t)s * plane + x0;
#pragma unroll
      for (int d = 1; d <= R; ++d) {
        float vm[4] = {0.0f, 0.0f, 0.0f, 0.0f}, vp[4] = {0.0f, 0.0f, 0.0f, 0.0f}, t[4];
        if (y == 0) {
          for (int i = 0; i <= min(d, a.ny - 1); ++i) {
            ld4(pl + (size_t)i * a.nx, t);
#pragma unroll
            for (int v = 0; v < 4; ++v) vm[v] += t[v];
          }
        } else if (y + d <= a.ny - 1) {
          ld4(pl + (size_t)(y + d) * a.nx, vm);
        }
        if (y == a.ny - 1) {
          for (int i = max(a.ny - 1 - d, 0); i <= a.ny - 1; ++i) {
            ld4(pl + (size_t)i * a.nx, t);
#pragma unroll
            for (int v = 0; v < 4; ++v) vp[v] += t[v];
          }
        } else if (y - d >= 0) {
          ld4(pl + (size_t)(y - d) * a.nx, vp);
        }
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          acc[v] = __builtin_fmaf(a.wm[1][d - 1], vm[v], acc[v]);
          acc[v] = __builtin_fmaf(a.wp[1][d - 1], vp[v], acc[v]);
        }
      }
    }
    // the marched axis from the window
#pragma unroll
    for (int d = 1; d <= R; ++d) {
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        float vm = win[R + d][v], vp = win[R - d][v];
        if (s == 0) {
          vm = 0.0f;
#pragma unroll
          for (int k = R; k <= R + d; ++k) vm += win[k][v];
        }
        if (s == ns - 1) {
          vp = 0.0f;
#pragma unroll
          for (int k = R - d; k <= R; ++k) vp += win[k][v];
        }
        acc[v] = __builtin_fmaf(a.wm[ma][d - 1], vm, acc[v]);
        acc[v] = __builtin_fmaf(a.wp[ma][d - 1], vp, acc[v]);
      }
    }
    const size_t cell = (size_t)s * st + roff + x0;
    store4(a.out + (size_t)s * st + roff, x0, a.nx, acc[0], acc[1], acc[2], acc[3], a.stream != 0);
    if (a.gp) {
      float g[4];
      ld4(a.gp + cell, g);
      *reinterpret_cast<float4*>(a.gp + cell) =
          make_float4(__builtin_fmaf(a.cp, win[R][0], g[0]), __builtin_fmaf(a.cp, win[R][1], g[1]),
                      __builtin_fmaf(a.cp, win[R][2], g[2]), __builtin_fmaf(a.cp, win[R][3], g[3]));
    }
#pragma unroll
    for (int k = 0; k < 2 * R; ++k)
#pragma unroll
      for (int v = 0; v < 4; ++v) win[k][v] = win[k + 1][v];
#pragma unroll
    for (int v = 0; v < 4; ++v) win[2 * R][v] = nxt[v];
  }
}

// Workgroups of one step: 256-cell pieces of x, by row (3D) and by kAdjMS-cell strip of the
// slowest axis (the same count for both kernels: 256 threads of one cell, or 64 of four).
inline long star_adjoint_blocks(const StarAdjArgs& a) {
  if (a.ndim == 3) return (long)a.nbx * a.ny * ((a.nz + kAdjMS - 1) / kAdjMS);
  return (long)a.nbx * ((a.ny + kAdjMS - 1) / kAdjMS);
}
