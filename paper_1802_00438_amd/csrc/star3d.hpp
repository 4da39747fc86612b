// star3d.hpp -- temporal-blocked radius-r 3D star stencil (diffusion form): 64 x 64 x-y
// windows streamed along z.
//
// Method (paper Eq. 1 and Eq. 2 with a general radius rad = R in 3D; Sections 3.1, 3.2): a cell
// is updated from itself and the cells at distance 1..R along x, y and z.  x-y tiles overlap
// by a halo of R*k cells per side, stream along z and fuse k time steps before writing back;
// per fused step the shift register of Eq. 1 spans 2R planes.
//
// gfx950 mapping:
//   * A workgroup of 16 wavefronts owns a 64 x 64 window; lane l of wave w holds column l of
//     rows 4w .. 4w+3 of every plane, so each row is one coalesced 256-byte access per wave.
//   * Level s (1..K) holds, per cell, the last R planes of level s-1 (the terms at z-d) and R
//     partial sums of its own pending planes (each still owed terms at z+d).  When level s-1
//     delivers plane q, every pending sum takes its next z+d term (plane q is z+1 for the
//     newest, z+R for the oldest, which is then complete) and plane q opens a new sum: centre,
//     x and y terms, then the z-d terms from the held planes.  The terms thus enter in the
//     order c, (w_d, e_d), s_d, n_d, b_d, a_d of the evaluation chain, and the R partial sums
//     take the place of the R planes ahead that a window of 2R+1 planes would hold.
//   * In-plane neighbours come from LDS: every level publishes its newest plane into a padded
//     (64+2R)^2 LDS plane, double-buffered by plane parity, so one barrier per plane serves
//     every level; level s consumes the plane that level s-1 published in the previous
//     iteration, so it runs R+1 planes behind level s-1.  y neighbours within a lane's own
//     four rows come from its registers.  Reads past the window edge land in the padding; they
//     feed only halo cells whose results are never stored.
//   * Clamp (Section 5.1, at every distance and every step): in tiles whose window reaches
//     past an x or y edge of the grid, the neighbour at distance d is replaced by the one at
//     distance d-1 where x-d (x+d, y-d, y+d) leaves the grid, which makes it the nearest
//     boundary cell.  Along z, a level sets every held plane to plane 0 when plane 0 arrives,
//     and takes its last held plane (plane nz-1) in place of planes past the top.
//   * A pass that fuses keff < K steps turns the levels past keff into delay lines of R planes.
#pragma once
#include "device_common.hpp"
#include "star2d.hpp"

struct Star3Coef {
  float c0;
  float w[kStarMaxR], e[kStarMaxR], s[kStarMaxR], n[kStarMaxR], b[kStarMaxR], a[kStarMaxR];
};

struct Star3dArgs {
  const float* src;
  float* dst;
  int nx, ny, nz;
  int keff;         // steps fused in this pass, 1..K
  int cs;           // output cells per tile in x and y (64 - 2*R*K)
  int ntx, nty;     // tiles along x and y
  int segz, nsegz;  // output planes per tile, tiles along z
  Star3Coef cf;
};

constexpr int kStar3W = 64;         // window width and height
constexpr int kStar3RY = 4;         // rows per lane
constexpr int kStar3Threads = 1024;  // 16 waves

constexpr int star3_lw(int R) { return kStar3W + 2 * R; }
// LDS floats of a (R, K) kernel: two parities x K levels x one padded plane
constexpr int star3_lds_floats(int R, int K) { return 2 * K * star3_lw(R) * star3_lw(R); }

template <int R, int K>
struct Star3dTile {
  static_assert(R >= 1 && R <= kStarMaxR, "radius");
  static constexpr int RY = kStar3RY;
  static constexpr int LW = star3_lw(R);
  static constexpr int PL = LW * LW;

  const Star3dArgs& a;
  float* lds;
  int gx, gy0, ox0, ox1, oy0, oy1, z0, z1, i0;
  int goff[RY];  // in-plane offsets of the lane's cells (clamped to the grid)
  int lidx;      // LDS index of the lane's first cell within one plane
  float hist[K][R][RY];  // level s: planes q-1 .. q-R of level s-1
  float pend[K][R][RY];  // level s: partial sums of its planes q-1 .. q-R (newest first)
  float out[K][RY];      // out[0]: the input plane; out[s]: level s's newest plane
  float lb[2][RY];       // input planes loaded two iterations ahead

  __device__ __forceinline__ Star3dTile(const Star3dArgs& args, float* l) : a(args), lds(l) {}

  __device__ __forceinline__ void load_plane(int z, float (&dstv)[RY]) const {
    const float* pl = a.src + (size_t)clampi(z, 0, a.nz - 1) * a.nx * a.ny;
#pragma unroll
    for (int j = 0; j < RY; ++j) dstv[j] = pl[goff[j]];
  }

  // New partial sum of plane q at level s from Q (level s-1's plane q, own cells), the
  // neighbours of that plane in LDS plane rp, and the held planes.
  template <bool EDGE>
  __device__ __forceinline__ void open_sum(int s, const float (&Q)[RY], const float* rp, float (&nw)[RY]) const {
#pragma unroll
    for (int j = 0; j < RY; ++j) {
      const float* cp = rp + lidx + j * LW;
      const float c = Q[j];
      const int gy = gy0 + j;
      float acc = a.cf.c0 * c;
      float vm = c, vp = c;
#pragma unroll
      for (int d = 1; d <= R; ++d) {
        float xm = cp[-d], xp = cp[d];
        if constexpr (EDGE) {
          xm = (gx - d >= 0) ? xm : vm;
          xp = (gx + d < a.nx) ? xp : vp;
          vm = xm;
          vp = xp;
        }
        acc = __builtin_fmaf(a.cf.w[d - 1], xm, acc);
        acc = __builtin_fmaf(a.cf.e[d - 1], xp, acc);
      }
      float v = c;
#pragma unroll
      for (int d = 1; d <= R; ++d) {
        float ys = (j + d < RY) ? Q[(j + d < RY) ? j + d : 0] : cp[d * LW];
        if constexpr (EDGE) {
          ys = (gy + d < a.ny) ? ys : v;
          v = ys;
        }
        acc = __builtin_fmaf(a.cf.s[d - 1], ys, acc);
      }
      v = c;
#pragma unroll
      for (int d = 1; d <= R; ++d) {
        float yn = (j - d >= 0) ? Q[(j - d >= 0) ? j - d : 0] : cp[-d * LW];
        if constexpr (EDGE) {
          yn = (gy - d >= 0) ? yn : v;
          v = yn;
        }
        acc = __builtin_fmaf(a.cf.n[d - 1], yn, acc);
      }
#pragma unroll
      for (int d = 1; d <= R; ++d) acc = __builtin_fmaf(a.cf.b[d - 1], hist[s - 1][d - 1][j], acc);
      nw[j] = acc;
    }
  }

  // Iteration it (input plane i = i0 + it arrives); P = it % 2 selects the LDS parity and the
  // load slot.
  template <int P, bool EDGE>
  __device__ __forceinline__ void iter(int it) {
    const int i = i0 + it;
    const float* rd = lds + (P ^ 1) * K * PL;  // planes published in the previous iteration
    float* wr = lds + P * K * PL;
    const size_t plane = (size_t)a.nx * a.ny;
    // top level first: level s reads out[s-1] before level s-1 replaces it
#pragma unroll
    for (int s = K; s >= 1; --s) {
      const int q = i - 1 - (s - 1) * (R + 1);  // plane of level s-1 that level s takes now
      if (q < 0) continue;                       // uniform: the pipeline is still filling
      const bool act = s <= a.keff;
      const bool past = q >= a.nz;
      float Q[RY];
#pragma unroll
      for (int j = 0; j < RY; ++j) Q[j] = past ? hist[s - 1][0][j] : out[s - 1][j];
      if (act) {
#pragma unroll
        for (int u = 0; u < R; ++u)
#pragma unroll
          for (int j = 0; j < RY; ++j) pend[s - 1][u][j] = __builtin_fmaf(a.cf.a[u], Q[j], pend[s - 1][u][j]);
      }
      float done[RY];
#pragma unroll
      for (int j = 0; j < RY; ++j) done[j] = pend[s - 1][R - 1][j];
      float nw[RY];
      if (!past) {
        if (q == 0) {
#pragma unroll
          for (int d = 0; d < R; ++d)
#pragma unroll
            for (int j = 0; j < RY; ++j) hist[s - 1][d][j] = Q[j];
        }
        if (act) {
          open_sum<EDGE>(s, Q, rd + (s - 1) * PL, nw);
        } else {
#pragma unroll
          for (int j = 0; j < RY; ++j) nw[j] = Q[j];
        }
#pragma unroll
        for (int d = R - 1; d >= 1; --d)
#pragma unroll
          for (int j = 0; j < RY; ++j) hist[s - 1][d][j] = hist[s - 1][d - 1][j];
#pragma unroll
        for (int j = 0; j < RY; ++j) hist[s - 1][0][j] = Q[j];
      } else {
#pragma unroll
        for (int j = 0; j < RY; ++j) nw[j] = Q[j];
      }
#pragma unroll
      for (int u = R - 1; u >= 1; --u)
#pragma unroll
        for (int j = 0; j < RY; ++j) pend[s - 1][u][j] = pend[s - 1][u - 1][j];
#pragma unroll
      for (int j = 0; j < RY; ++j) pend[s - 1][0][j] = nw[j];
      if (s < K) {
#pragma unroll
        for (int j = 0; j < RY; ++j) {
          out[s][j] = done[j];
          wr[s * PL + lidx + j * LW] = done[j];
        }
      } else {
        const int p = q - R;  // the plane level K completes now
        if (p >= z0 && p < z1 && gx >= ox0 && gx < ox1) {
          float* dp = a.dst + (size_t)p * plane;
#pragma unroll
          for (int j = 0; j < RY; ++j) {
            const int gy = gy0 + j;
            if (gy >= oy0 && gy < oy1) dp[(size_t)gy * a.nx + gx] = done[j];
          }
        }
      }
    }
    // level 0: publish input plane i, load plane i + 2 into the freed slot
#pragma unroll
    for (int j = 0; j < RY; ++j) {
      out[0][j] = lb[P][j];
      wr[lidx + j * LW] = lb[P][j];
    }
    load_plane(i + 2, lb[P]);
    __syncthreads();
  }

  template <bool EDGE>
  __device__ __forceinline__ void run() {
    const int nit = (z1 - z0) + K * (2 * R + 1);
    for (int it = 0; it < nit; it += 2) {
      iter<0, EDGE>(it);
      iter<1, EDGE>(it + 1);  // one surplus iteration when nit is odd: it stores nothing
    }
  }

  __device__ __forceinline__ void process(int tile) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int tx = tile % a.ntx;
    const int t2 = tile / a.ntx;
    const int ty = t2 % a.nty;
    const int sz = t2 / a.nty;
    ox0 = tx * a.cs;
    oy0 = ty * a.cs;
    ox1 = min(ox0 + a.cs, a.nx);
    oy1 = min(oy0 + a.cs, a.ny);
    const int xw = ox0 - R * K, yw = oy0 - R * K;
    gx = xw + lane;
    gy0 = yw + wave * RY;
    z0 = sz * a.segz;
    z1 = min(z0 + a.segz, a.nz);
    i0 = z0 - R * K;
    lidx = (wave * RY + R) * LW + lane + R;
#pragma unroll
    for (int j = 0; j < RY; ++j) goff[j] = clampi(gy0 + j, 0, a.ny - 1) * a.nx + clampi(gx, 0, a.nx - 1);
#pragma unroll
    for (int s = 0; s < K; ++s)
#pragma unroll
      for (int j = 0; j < RY; ++j) {
        out[s][j] = 0.0f;
#pragma unroll
        for (int d = 0; d < R; ++d) {
          hist[s][d][j] = 0.0f;
          pend[s][d][j] = 0.0f;
        }
      }
    load_plane(i0, lb[0]);
    load_plane(i0 + 1, lb[1]);
    const bool edge = (xw < 0) || (xw + kStar3W > a.nx) || (yw < 0) || (yw + kStar3W > a.ny);
    if (edge) run<true>();
    else run<false>();
  }
};

template <int R, int K>
__global__ __launch_bounds__(kStar3Threads) void star3d_kernel(Star3dArgs a) {
  __shared__ float lds[star3_lds_floats(R, K)];
  const int tile = xcd_remap(blockIdx.x, gridDim.x);
  Star3dTile<R, K> t(a, lds);
  t.process(tile);
}
