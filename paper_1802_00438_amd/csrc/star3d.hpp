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
//     (64+2R)^2 LDS plane, in one of three buffers taken in turn, so one barrier per plane
//     serves every level; level s consumes the plane that level s-1 published in the previous
//     iteration, so it runs R+1 planes behind level s-1.  Input planes land in three register
//     slots, loaded two planes ahead; the loop is unrolled by three so that every slot and LDS
//     buffer is a fixed register set or address and no load result is copied (a copy would
//     wait for the load at once).  y neighbours within a lane's own four rows come from its
//     registers.  Reads past the window edge land in the padding; they feed only halo cells
//     whose results are never stored.
//   * Clamp (Section 5.1, at every distance and every step): in tiles whose window reaches
//     past an x or y edge of the grid, the neighbour at distance d is replaced by the one at
//     distance d-1 where x-d (x+d, y-d, y+d) leaves the grid, which makes it the nearest
//     boundary cell.  Along z, a level sets every held plane to plane 0 when plane 0 arrives,
//     and takes its last held plane (plane nz-1) in place of planes past the top.
//   * Every step count from 1 to the largest k is instantiated, so a pass always runs on the
//     kernel whose K equals the steps it fuses.
//   * Hotspot form (HOT): a new sum starts from fma(cc, c, q) with q = fma(cp, p, kamb) of its
//     own plane and cell, as the radius-1 hotspot does; each level reads the power plane of the
//     plane it opens (the same plane for every level, one iteration apart, so an L2 hit after
//     the first).
#pragma once
#include "device_common.hpp"
#include "star2d.hpp"

struct Star3Coef {
  float c0;
  float w[kStarMaxR], e[kStarMaxR], s[kStarMaxR], n[kStarMaxR], b[kStarMaxR], a[kStarMaxR];
  float cp, kamb;  // hotspot form: q = fma(cp, p, kamb), kamb = c_amb * t_amb rounded in FP32
};

struct Star3dArgs {
  const float* src;
  float* dst;
  const float* power;  // hotspot form: the power map (grid shape); diffusion: unused
  int nx, ny, nz;
  int keff;         // steps fused in this pass (equal to K)
  int cs;           // output cells per tile in x and y (64 - 2*R*K)
  int ntx, nty;     // tiles along x and y
  int segz, nsegz;  // output planes per tile, tiles along z
  Star3Coef cf;
};

constexpr int kStar3W = 64;         // window width and height
constexpr int kStar3RY = 4;         // rows per lane
constexpr int kStar3Threads = 1024;  // 16 waves

constexpr int star3_lw(int R) { return kStar3W + 2 * R; }
constexpr int star3_gcd(int a, int b) { return b == 0 ? a : star3_gcd(b, a % b); }
constexpr int star3_lcm(int a, int b) { return a / star3_gcd(a, b) * b; }
// LDS floats of a (R, K) kernel: three buffers x K levels x one padded plane
constexpr int star3_lds_floats(int R, int K) { return 3 * K * star3_lw(R) * star3_lw(R); }

template <int R, int K, bool HOT>
struct Star3dTile {
  static_assert(R >= 1 && R <= kStarMaxR, "radius");
  static constexpr int RY = kStar3RY;
  static constexpr int LW = star3_lw(R);
  static constexpr int PL = LW * LW;

  const Star3dArgs& a;
  float* lds;
  int gx, gy0, ox0, ox1, oy0, oy1, z0, z1, i0;
  unsigned goff[RY];  // in-plane byte offsets of the lane's cells (clamped to the grid)
  int lidx;      // LDS index of the lane's first cell within one plane
  // Rings addressed by the iteration phase u (it mod U, a compile-time constant):
  //   hist[s-1][(u - d) mod HS]: plane q-d of level s-1 (d = 1..R); plane q goes to slot u mod HS
  //   pend[s-1][(u - j) mod PS]: level s's partial sum of plane q-j (j = 0..R); the sum of
  //   plane q-R completes in iteration u and stays in its slot through iteration u+1, where
  //   level s+1 takes it as its input plane (so PS = R+1 when a level above reads it).
  static constexpr int HS = R;
  static constexpr int PS = K > 1 ? R + 1 : R;
  static constexpr int U = star3_lcm(3, star3_lcm(HS, PS));
  float hist[K][HS][RY];
  float pend[K][PS][RY];
  float lb[3][RY];  // input planes i-1, i, i+1 (plane i0 + it in slot it mod 3)

  __device__ __forceinline__ Star3dTile(const Star3dArgs& args, float* l) : a(args), lds(l) {}

  // (a uniform plane base plus 32-bit lane offsets: the loads take the scalar-base form)
  __device__ __forceinline__ void load_plane(int z, float (&dstv)[RY]) const {
    const char* pl = reinterpret_cast<const char*>(a.src + (size_t)clampi(z, 0, a.nz - 1) * a.nx * a.ny);
#pragma unroll
    for (int j = 0; j < RY; ++j) dstv[j] = *reinterpret_cast<const float*>(pl + goff[j]);
  }

  // New partial sum of plane q at level s from Q (level s-1's plane q, own cells), the
  // neighbours of that plane in LDS plane rp, and the held planes.
  template <int u, bool EDGE>
  __device__ __forceinline__ void open_sum(int s, int qz, const float (&Q)[RY], const float* rp,
                                           float (&nw)[RY]) const {
    float src[RY];
    if constexpr (HOT) {
      const char* pp = reinterpret_cast<const char*>(a.power + (size_t)qz * a.nx * a.ny);
#pragma unroll
      for (int j = 0; j < RY; ++j)
        src[j] = __builtin_fmaf(a.cf.cp, *reinterpret_cast<const float*>(pp + goff[j]), a.cf.kamb);
    }
#pragma unroll
    for (int j = 0; j < RY; ++j) {
      const float* cp = rp + lidx + j * LW;
      const float c = Q[j];
      const int gy = gy0 + j;
      float acc = HOT ? __builtin_fmaf(a.cf.c0, c, src[j]) : a.cf.c0 * c;
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
      for (int d = 1; d <= R; ++d) acc = __builtin_fmaf(a.cf.b[d - 1], hist[s - 1][(u - d + 4 * HS) % HS][j], acc);
      nw[j] = acc;
    }
  }

  // Iteration it (input plane i = i0 + it arrives) at phase u = it mod U; P = u mod 3 selects
  // the LDS buffer written and the load slot of plane i.  TOP: some level may be past the top
  // plane (q >= nz), which only the last iterations of a tile can be.
  template <int u, bool EDGE, bool TOP>
  __device__ __forceinline__ void iter(int it) {
    constexpr int P = u % 3, PP = (P + 2) % 3;  // PP: the previous iteration's buffer, plane i-1's slot
    constexpr int SH = u % HS, SP = u % PS;
    const int i = i0 + it;
    const float* rd = lds + PP * K * PL;  // planes published in the previous iteration
    float* wr = lds + P * K * PL;
    const size_t plane = (size_t)a.nx * a.ny;
    // top level first: level s takes level s-1's plane completed in the previous iteration
    // before level s-1 runs
#pragma unroll
    for (int s = K; s >= 1; --s) {
      const int q = i - 1 - (s - 1) * (R + 1);  // plane of level s-1 that level s takes now
      if (q < 0) continue;                       // uniform: the pipeline is still filling
      const bool past = TOP && q >= a.nz;
      float Q[RY];
#pragma unroll
      for (int j = 0; j < RY; ++j) {
        // level s-1's plane completed in iteration it-1: its slot (u-1-R) mod PS = u mod PS
        const float v = s == 1 ? lb[PP][j] : pend[s > 1 ? s - 2 : 0][SP][j];
        Q[j] = past ? hist[s - 1][(u - 1 + HS) % HS][j] : v;  // past the top: plane nz-1
      }
#pragma unroll
      for (int t = 0; t < R; ++t)  // plane q is z+1+t of the sum of plane q-1-t
#pragma unroll
        for (int j = 0; j < RY; ++j) {
          float& ps = pend[s - 1][(u - 1 - t + 4 * PS) % PS][j];
          ps = __builtin_fmaf(a.cf.a[t], Q[j], ps);
        }
      constexpr int SD = (u - R + 4 * PS) % PS;  // the sum of plane q-R, complete now
      if (s == K) {
        const int p = q - R;
        if (p >= z0 && p < z1 && gx >= ox0 && gx < ox1) {
          // an output cell is inside the grid, where goff is its unclamped offset
          char* dp = reinterpret_cast<char*>(a.dst + (size_t)p * plane);
#pragma unroll
          for (int j = 0; j < RY; ++j) {
            const int gy = gy0 + j;
            if (gy >= oy0 && gy < oy1) *reinterpret_cast<float*>(dp + goff[j]) = pend[s - 1][SD][j];
          }
        }
      } else {
#pragma unroll
        for (int j = 0; j < RY; ++j) wr[s * PL + lidx + j * LW] = pend[s - 1][SD][j];
      }
      if (!past) {
        if (q == 0) {
#pragma unroll
          for (int d = 0; d < HS; ++d)
#pragma unroll
            for (int j = 0; j < RY; ++j) hist[s - 1][d][j] = Q[j];
        }
        float nw[RY];
        open_sum<u, EDGE>(s, q, Q, rd + (s - 1) * PL, nw);
#pragma unroll
        for (int j = 0; j < RY; ++j) {
          pend[s - 1][SP][j] = nw[j];
          hist[s - 1][SH][j] = Q[j];
        }
      } else {
#pragma unroll
        for (int j = 0; j < RY; ++j) {
          pend[s - 1][SP][j] = Q[j];
          hist[s - 1][SH][j] = Q[j];  // the newest slot keeps plane nz-1
        }
      }
    }
    // level 0: publish input plane i; plane i+2 goes to the slot of plane i-1, which level 1
    // has just consumed
#pragma unroll
    for (int j = 0; j < RY; ++j) wr[lidx + j * LW] = lb[P][j];
    load_plane(i + 2, lb[PP]);
    __syncthreads();
  }

  template <int u, bool EDGE, bool TOP>
  __device__ __forceinline__ void iters(int it) {
    if constexpr (u < U) {
      iter<u, EDGE, TOP>(it + u);
      iters<u + 1, EDGE, TOP>(it);
    }
  }

  template <bool EDGE>
  __device__ __forceinline__ void run() {
    const int nit = (z1 - z0) + K * (2 * R + 1);
    // iterations it with i0 + it - 1 < nz have every level below the top plane
    const int nlow = min(nit, a.nz + 1 - i0);
    int it = 0;
    for (; it + U <= nlow; it += U) iters<0, EDGE, false>(it);
    for (; it < nit; it += U) iters<0, EDGE, true>(it);  // surplus iterations store nothing
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
    for (int j = 0; j < RY; ++j)
      goff[j] = 4u * (unsigned)(clampi(gy0 + j, 0, a.ny - 1) * a.nx + clampi(gx, 0, a.nx - 1));
#pragma unroll
    for (int s = 0; s < K; ++s)
#pragma unroll
      for (int j = 0; j < RY; ++j) {
#pragma unroll
        for (int d = 0; d < HS; ++d) hist[s][d][j] = 0.0f;
#pragma unroll
        for (int d = 0; d < PS; ++d) pend[s][d][j] = 0.0f;
      }
    load_plane(i0, lb[0]);
    load_plane(i0 + 1, lb[1]);
#pragma unroll
    for (int j = 0; j < RY; ++j) lb[2][j] = 0.0f;  // "plane i0-1": level 1 takes nothing before i0
    const bool edge = (xw < 0) || (xw + kStar3W > a.nx) || (yw < 0) || (yw + kStar3W > a.ny);
    if (edge) run<true>();
    else run<false>();
  }
};

template <int R, int K, bool HOT>
__global__ __launch_bounds__(kStar3Threads) void star3d_kernel(Star3dArgs a) {
  __shared__ float lds[star3_lds_floats(R, K)];
  const int tile = xcd_remap(blockIdx.x, gridDim.x);
  Star3dTile<R, K, HOT> t(a, lds);
  t.process(tile);
}
