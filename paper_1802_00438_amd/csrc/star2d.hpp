// star2d.hpp -- temporal-blocked radius-r 2D star stencil (diffusion and hotspot forms), one
// wave per tile.
//
// Method (paper Eq. 1 and Eq. 2 with a general radius rad = R; Sections 3.1, 3.2): a cell is
// updated from itself and the cells at distance 1..R along x and y.  Tiles overlap by a halo
// of R*k cells per side, stream along y and fuse k time steps before writing back.
//
// gfx950 mapping:
//   * One 64-lane wavefront owns a 256-column window, 4 consecutive cells per lane (one
//     16-byte access per row).  x-neighbours at distance d <= 4 are in the lane itself or,
//     for the first / last d cells, in the lower / upper lane, read through DPP; in tiles away
//     from the x edges that read is fused into the multiply-add (v_fmac_f32_dpp).
//   * Level s (1..K) keeps the last 2R+1 rows of level s-1 in registers.  When level s-1
//     produces row i, level s computes row i+R (centre, x-terms, then the R rows below and the
//     R rows above), so level s trails level s-1 by R rows.  The row loop is unrolled by 2R+1,
//     which makes every window slot a compile-time register set.
//   * Only the last term (the row R above, which level s-1 produces in the same step) depends
//     on this step's work of the level below.  Away from the first and last grid rows, each
//     step therefore runs in two phases: every level sums all its other terms (independent
//     work across levels) into the window slot its new row will occupy, which is free; then,
//     bottom level first, each adds the last term.  Tiles near the first or last row, whose
//     row clamp may substitute that term, evaluate each level in one go.
//   * Clamp (Section 5.1 at every distance): an index beyond the grid is the nearest
//     boundary index.  For a cell at x, the clamped neighbour at distance d is its neighbour at
//     distance min(d, x) (left) or min(d, nx-1-x) (right), so edge tiles select, per
//     distance, between the neighbour and the previous distance's value; rows likewise, with
//     a row-uniform condition.  Tiles away from every edge compile no selects.
//   * Evaluation order, the same FMA chain as the oracle: acc = cc*c; for d = 1..R:
//     acc = fma(w_d, x-d, acc), acc = fma(e_d, x+d, acc); then fma(s_d, y+d) for d = 1..R,
//     then fma(n_d, y-d) for d = 1..R.
//   * Hotspot form (HOT): the chain starts from fma(cc, c, q), q = fma(cp, p, kamb) of the
//     cell, as the radius-1 hotspot does.  Each level reads the power row of the row it makes
//     (the rows of the K levels are K*R rows apart, so all but the first read hit L2).
#pragma once
#include "device_common.hpp"

constexpr int kStarMaxR = 4;

struct StarCoef {
  float c0;
  float w[kStarMaxR], e[kStarMaxR], s[kStarMaxR], n[kStarMaxR];
  float cp, kamb;  // hotspot form: q = fma(cp, p, kamb), kamb = c_amb * t_amb rounded in FP32
};

struct Star2dArgs {
  const float* src;
  float* dst;
  const float* power;  // hotspot form: the power map (grid shape); diffusion: unused
  int nx, ny;
  int keff;  // steps fused in this pass, 1..K
  int cs;    // output columns per tile (multiple of 4)
  int kr;    // left halo of the window (>= R*K, multiple of 4)
  int ntx;   // tiles along x
  int seg;   // output rows per tile
  int nseg;  // tiles along y
  int aligned;  // nx % 4 == 0 and 16-byte aligned buffers: vector loads and stores
  StarCoef cf;
};

// FULL: the pass fuses all K steps (keff == K), so no level needs the run-time keff test that
// would split the unrolled step into one basic block per level.
template <int R, int K, bool FULL, bool HOT = false>
struct Star2dTile {
  static_assert(R >= 1 && R <= kStarMaxR, "radius");
  static constexpr int V = 4;
  static constexpr int W = 64 * V;
  static constexpr int NR = 2 * R + 1;  // rows of a level's window; also the loop unroll

  const Star2dArgs& a;
  const int lane;
  int ws, ox0, ox1, y0, y1;
  float win[K][NR][V];  // win[s]: the last NR rows of level s (s = 0: input rows), by arrival slot
  float Lb[NR][V];      // input rows in flight: the row of step t is loaded NR steps ahead, into slot t % NR
  int xl[V];            // column of each of the lane's cells

  __device__ __forceinline__ Star2dTile(const Star2dArgs& args, int ln) : a(args), lane(ln) {}

  template <bool VEC>
  __device__ __forceinline__ void load_row(int r, float (&dstv)[V]) const {
    const int jr = clampi(r, 0, a.ny - 1);
    const float* rowp = a.src + (size_t)jr * a.nx;
    const int x0 = ws + lane * V;
    if constexpr (VEC) {
      const float4 t = *reinterpret_cast<const float4*>(rowp + x0);
      dstv[0] = t.x; dstv[1] = t.y; dstv[2] = t.z; dstv[3] = t.w;
    } else {
#pragma unroll
      for (int v = 0; v < V; ++v) dstv[v] = rowp[clampi(x0 + v, 0, a.nx - 1)];
    }
  }

  template <bool VEC>
  __device__ __forceinline__ void store_row(int j, const float (&o)[V], bool xe) const {
    float* rowp = a.dst + (size_t)j * a.nx;
    const int x0 = ws + lane * V;
    if (VEC && !xe) {
      if (x0 >= ox0 && x0 < ox1) *reinterpret_cast<float4*>(rowp + x0) = make_float4(o[0], o[1], o[2], o[3]);
    } else {
#pragma unroll
      for (int v = 0; v < V; ++v)
        if (x0 + v >= ox0 && x0 + v < ox1) rowp[x0 + v] = o[v];
    }
  }

  // q = fma(cp, p, kamb) of the lane's cells of row j (clamped, so a halo row outside the grid
  // reads a valid address; its results are never stored)
  template <bool XE, bool VEC>
  __device__ __forceinline__ void source_row(int j, float (&q)[V]) const {
    const float* rowp = a.power + (size_t)clampi(j, 0, a.ny - 1) * a.nx;
    const int x0 = ws + lane * V;
    if constexpr (VEC && !XE) {
      const float4 t = *reinterpret_cast<const float4*>(rowp + x0);
      q[0] = t.x; q[1] = t.y; q[2] = t.z; q[3] = t.w;
    } else {
#pragma unroll
      for (int v = 0; v < V; ++v) q[v] = rowp[clampi(x0 + v, 0, a.nx - 1)];
    }
#pragma unroll
    for (int v = 0; v < V; ++v) q[v] = __builtin_fmaf(a.cf.cp, q[v], a.cf.kamb);
  }

  // Row j of level s from the window P of level s-1, whose newest row (slot NW) is row j - R.
  // The row that arrived u steps ago sits in slot (NW - u) mod NR and is row j - R + u.  With
  // LAST = false the final term (n_R times the newest row) is left out.
  template <bool XE, bool YE, int NW, bool LAST = true, bool VEC = false>
  __device__ __forceinline__ void level_row(const float (&P)[NR][V], int j, float (&o)[V]) const {
    constexpr int CS = (NW - R + 2 * NR) % NR;  // centre slot (u = R)
    const float(&C)[V] = P[CS];
    float q[V];
    if constexpr (HOT) source_row<XE, VEC>(j, q);
    // x-neighbours: xm[d][v] is the value at distance d to the left of cell v, xp to the right
    float xm[R + 1][V], xp[R + 1][V];
    float lo[R], up[R];
#pragma unroll
    for (int d = 0; d < R; ++d) {
      lo[d] = from_lower(C[V - 1 - d]);  // lane-1's cell V-1-d
      up[d] = from_upper(C[d]);          // lane+1's cell d
    }
#pragma unroll
    for (int v = 0; v < V; ++v) {
      xm[0][v] = C[v];
      xp[0][v] = C[v];
#pragma unroll
      for (int d = 1; d <= R; ++d) {
        const int im = v - d, ip = v + d;
        float vm = im >= 0 ? C[im >= 0 ? im : 0] : lo[(-im - 1) < R ? (-im - 1) : 0];
        float vp = ip < V ? C[ip < V ? ip : 0] : up[(ip - V) < R ? (ip - V) : 0];
        if constexpr (XE) {
          vm = (xl[v] - d >= 0) ? vm : xm[d - 1][v];
          vp = (xl[v] + d <= a.nx - 1) ? vp : xp[d - 1][v];
        }
        xm[d][v] = vm;
        xp[d][v] = vp;
      }
    }
    // y-neighbours: rows j+d (below, slot u = R+d) and j-d (above, u = R-d), clamped
    float ys[R + 1][V], yn[R + 1][V];
#pragma unroll
    for (int v = 0; v < V; ++v) {
      ys[0][v] = C[v];
      yn[0][v] = C[v];
    }
#pragma unroll
    for (int d = 1; d <= R; ++d) {
      const int ss = (NW - (R + d) + 2 * NR) % NR;
      const int sn = (NW - (R - d) + 2 * NR) % NR;
      bool okS = true, okN = true;
      if constexpr (YE) {
        okS = (j + d <= a.ny - 1);
        okN = (j - d >= 0);
      }
#pragma unroll
      for (int v = 0; v < V; ++v) {
        ys[d][v] = okS ? P[ss][v] : ys[d - 1][v];
        yn[d][v] = okN ? P[sn][v] : yn[d - 1][v];
      }
    }
#pragma unroll
    for (int v = 0; v < V; ++v) {
      float acc = HOT ? __builtin_fmaf(a.cf.c0, C[v], q[v]) : a.cf.c0 * C[v];
#pragma unroll
      for (int d = 1; d <= R; ++d) {
        const int im = v - d, ip = v + d;
        if constexpr (!XE) {
          // a neighbour in the next lane: the move is fused into the multiply-add
          if (im < 0) acc = fma_from_lower_dpp(a.cf.w[d - 1], C[(V - 1 - (-im - 1)) & (V - 1)], acc);
          else acc = __builtin_fmaf(a.cf.w[d - 1], xm[d][v], acc);
          if (ip >= V) acc = fma_from_upper_dpp(a.cf.e[d - 1], C[(ip - V) & (V - 1)], acc);
          else acc = __builtin_fmaf(a.cf.e[d - 1], xp[d][v], acc);
        } else {
          acc = __builtin_fmaf(a.cf.w[d - 1], xm[d][v], acc);
          acc = __builtin_fmaf(a.cf.e[d - 1], xp[d][v], acc);
        }
      }
#pragma unroll
      for (int d = 1; d <= R; ++d) acc = __builtin_fmaf(a.cf.s[d - 1], ys[d][v], acc);
#pragma unroll
      for (int d = 1; d <= (LAST ? R : R - 1); ++d) acc = __builtin_fmaf(a.cf.n[d - 1], yn[d][v], acc);
      o[v] = acc;
    }
  }

  // One row step (slot T of the unrolled loop): input row r arrives; level s makes row r + sR.
  template <int T, bool XE, bool YE, bool VEC>
  __device__ __forceinline__ void step(int r) {
#pragma unroll
    for (int v = 0; v < V; ++v) win[0][T][v] = Lb[T][v];
    load_row<VEC>(r - NR, Lb[T]);
    if constexpr (!YE) {
      constexpr int CS = (T - R + 2 * NR) % NR;
      // phase 1, top level first: all terms but the last, into slot T of the level's own
      // window (its previous occupant, 2R+1 rows old, is dead)
      float top[V];
#pragma unroll
      for (int s = K; s >= 1; --s) {
        float o[V];
        if (FULL || s <= a.keff) {
          level_row<XE, false, T, false, VEC>(win[s - 1], r + s * R, o);
        } else {
#pragma unroll
          for (int v = 0; v < V; ++v) o[v] = 0.0f;  // surplus level: set in phase 2
        }
#pragma unroll
        for (int v = 0; v < V; ++v) {
          if (s == K) top[v] = o[v];
          else win[s][T][v] = o[v];
        }
      }
      // phase 2, bottom level first: the last term, from the row level s-1 has just made
#pragma unroll
      for (int s = 1; s <= K; ++s) {
        const int j = r + s * R;
        float o[V];
        if (FULL || s <= a.keff) {
#pragma unroll
          for (int v = 0; v < V; ++v)
            o[v] = __builtin_fmaf(a.cf.n[R - 1], win[s - 1][T][v], s == K ? top[v] : win[s][T][v]);
        } else {
#pragma unroll
          for (int v = 0; v < V; ++v) o[v] = win[s - 1][CS][v];  // surplus level: forward its input
        }
        if (s < K) {
#pragma unroll
          for (int v = 0; v < V; ++v) win[s][T][v] = o[v];
        } else if (j >= y0 && j < y1) {
          store_row<VEC>(j, o, XE);
        }
      }
      return;
    }
#pragma unroll
    for (int s = 1; s <= K; ++s) {
      const int j = r + s * R;
      float o[V];
      if (FULL || s <= a.keff) {
        level_row<XE, YE, T, true, VEC>(win[s - 1], j, o);
      } else {
        // levels past keff forward their input row (the centre of the window below)
        constexpr int CS = (T - R + 2 * NR) % NR;
#pragma unroll
        for (int v = 0; v < V; ++v) o[v] = win[s - 1][CS][v];
      }
      if (s < K) {
#pragma unroll
        for (int v = 0; v < V; ++v) win[s][T][v] = o[v];
      } else if (j >= y0 && j < y1) {
        store_row<VEC>(j, o, XE);
      }
    }
  }

  template <int T, bool XE, bool YE, bool VEC>
  __device__ __forceinline__ void steps(int r) {
    if constexpr (T < NR) {
      step<T, XE, YE, VEC>(r - T);
      steps<T + 1, XE, YE, VEC>(r);
    }
  }

  template <bool XE, bool YE, bool VEC>
  __device__ __forceinline__ void run() {
#pragma unroll
    for (int s = 0; s < K; ++s)
#pragma unroll
      for (int b = 0; b < NR; ++b)
#pragma unroll
        for (int v = 0; v < V; ++v) win[s][b][v] = 0.0f;
    // input rows from y1-1+K*R down to y0-K*R; level K emits row r + K*R, the first valid
    // one once every level's window has filled (2R steps per level)
    const int r0 = y1 - 1 + K * R;
    int nit = (y1 - y0) + 2 * K * R;
    nit = (nit + NR - 1) / NR * NR;  // the extra steps only touch rows outside [y0, y1)
#pragma unroll
    for (int b = 0; b < NR; ++b) load_row<VEC>(r0 - b, Lb[b]);
    for (int it = 0; it < nit; it += NR) steps<0, XE, YE, VEC>(r0 - it);
  }

  __device__ __forceinline__ void process(int tile) {
    const int tx = tile % a.ntx;
    const int sg = tile / a.ntx;
    ox0 = tx * a.cs;
    ox1 = min(ox0 + a.cs, a.nx);
    ws = ox0 - a.kr;
    y0 = sg * a.seg;
    y1 = min(y0 + a.seg, a.ny);
#pragma unroll
    for (int v = 0; v < V; ++v) xl[v] = ws + lane * V + v;
    const bool xe = (ws < 0) || (ws + W > a.nx);
    const bool ye = (y0 - K * R <= 0) || (y1 + K * R >= a.ny);
    if (xe) {
      if (ye) run<true, true, false>(); else run<true, false, false>();
    } else if (a.aligned) {
      if (ye) run<false, true, true>(); else run<false, false, true>();
    } else {
      if (ye) run<false, true, false>(); else run<false, false, false>();
    }
  }
};

// Radius 2 with five fused steps sits a few registers above the three-waves-per-SIMD limit
// (168); the diffusion form is held to that limit (a 12-byte spill).  The hotspot form needs
// more (the power row in flight), and held to 168 it would spill 356 bytes, so it is not.
// Everything else takes what the compiler allocates.
constexpr int star_min_waves(int R, int K, bool HOT) { return (!HOT && R == 2 && K == 5) ? 3 : 1; }

template <int R, int K, bool FULL, bool HOT>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(star_min_waves(R, K, HOT))))
void star2d_kernel(Star2dArgs a) {
  const int tile = xcd_remap(blockIdx.x, gridDim.x);
  Star2dTile<R, K, FULL, HOT> t(a, threadIdx.x);
  t.process(tile);
}
