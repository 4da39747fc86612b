// tb2d.hpp -- temporal-blocked 2D star stencil, one wavefront per overlapped tile.
//
// Method (paper Sections 3.1, 3.2; Eq. 2, Eq. 4, Eq. 5): the grid is cut into spatial blocks
// along x that overlap by a halo of k cells per side (k = fused time steps of one pass); each
// block streams along y and applies k consecutive time steps before anything goes back to
// memory.  Step s of the block trails step s-1 by one row, so no block ever waits for
// another; halo cells are computed redundantly and only the compute block is stored.
//
// gfx950 mapping (not the paper's FPGA pipeline):
//   * One 64-lane wavefront owns a window of 64*V columns; lane l holds columns
//     [ws + l*V, ws + l*V + V) of every row it touches, so each row of the window is one
//     16-byte vector access per lane (coalesced, aligned when nx % 4 == 0).
//   * The tile streams its rows bottom-up.  Level s (1..K) computes row r+s while level 0
//     receives row r, from rows r+s+1 (below, y+1), r+s (centre) and r+s-1 (above, y-1) of
//     level s-1.  The canonical term order (centre, x-1, x+1, y+1, y-1) puts the row that
//     arrived first (y+1) before the row that arrives last (y-1), so each iteration runs in
//     two phases: (1) for every level, fold the centre row and the oldest row into a partial
//     sum, which frees the oldest row's registers; (2) walking up the levels, add the y-1
//     term from the row the level below has just produced.  Each level therefore keeps two
//     rows in registers (centre, and oldest/partial/newest in turn) -- the register analogue
//     of the paper's shift register (Eq. 1) -- and the row loop, unrolled by two, renames
//     them without copies.
//   * x-neighbours across lanes come from DPP wave shifts; no LDS traffic is needed for the
//     temperature field.
//   * Hotspot: the time-invariant source q = fma(cp, p, kamb) of each row is formed once
//     when the power row arrives and parked in a per-wave LDS ring of k+1 rows, from which
//     each of the k levels reads it.
//   * Clamp-to-edge (Section 5.1) is applied at every fused level by substituting the
//     cell's own value for an out-of-grid neighbour.  Tiles that touch no grid edge take a
//     code path with no boundary code at all (wave-uniform dispatch).
//   * Adjoint mode applies the transposed operator: mirrored weights, zero contribution
//     from outside the grid, and a self term with the weight of the direction that leaves
//     the grid; sum_s lambda_s is carried along the level pipeline and added to grad_p once
//     per pass.
//   * Passes with fewer than K steps (the tail of T, Section 3.2) run the same kernel with
//     the levels past keff simply forwarding their input row.
//   * PHYS: Table 2's Hotspot 2D as printed, c + sdc*(p + ((n+s)-2c)*Ry_1 + ((e+w)-2c)*Rx_1
//     + (TEMP_AMB-c)*Rz_1), each operation rounded in that order.  Its first operation needs
//     the oldest and the newest row together, so phase 1 keeps the oldest row in place of a
//     partial sum (same registers) and phase 2 evaluates the whole formula; the ring holds the
//     raw power rows.  Its linear part has equal weights on both sides of each axis, so with
//     the clamp it is a symmetric matrix: the transposed step (ADJ) is the same formula with
//     no power and TEMP_AMB = 0.
#pragma once
#include "device_common.hpp"

// Rows of the hotspot source ring: at least K+1.  Rounded up to a power of two (the slot
// index becomes a mask instead of a compare-and-select per level) when that wastes less than
// a third of the ring.  For K = 12 that is 16 rows: 10 workgroups per CU instead of the 12 a
// 13-row ring admits, yet measured 2% faster than the 13-row ring.
constexpr int tb2d_ring_rows(int K) {
  int p = 1;
  while (p < K + 1) p *= 2;
  return 3 * p <= 4 * (K + 1) ? p : K + 1;
}

struct Tb2dArgs {
  const float* src;
  float* dst;
  const float* power;  // forward hotspot only
  float* gp;           // adjoint hotspot: grad_p accumulator (read-modify-write); else null
  int nx, ny;
  int keff;            // steps fused in this pass, 1..K
  int cs;              // output columns per tile (multiple of 4)
  int kr;              // left halo of the window (>= K, multiple of 4)
  int ntx;             // tiles along x
  int seg;             // output rows per tile
  int nseg;            // tiles along y
  int aligned;         // 1: nx % 4 == 0 and 16-byte aligned buffers (vector access in interior tiles)
  int stream;          // 1: nontemporal vector stores of the output (grids far larger than the cache)
  // Tiles of this launch: part 0 = every tile; part 1 = the interior rectangle
  // [ix0, ix1) x [iy0, iy1) of tiles that touch no grid edge; part 2 = the frame of all others.
  int part, ix0, ix1, iy0, iy1;
  // Output rows [ylo, yhi) of the streamed axis; tile segments start at ylo.  Every row
  // normally; a slab pass with ghost rows stores only the rows between them.
  int ylo, yhi;
  DevCoef cf;
};

// Tile id of the i-th tile of the launch's part.
__device__ __forceinline__ int tb2d_part_tile(const Tb2dArgs& a, int i) {
  const int w = a.ix1 - a.ix0;
  if (a.part == 1) return (a.iy0 + i / w) * a.ntx + a.ix0 + i % w;
  if (a.part == 2) {
    const int ntop = a.iy0 * a.ntx, nmid = (a.iy1 - a.iy0) * (a.ntx - w);
    if (i < ntop) return i;
    if (i < ntop + nmid) {
      const int j = i - ntop, c = j % (a.ntx - w);
      return (a.iy0 + j / (a.ntx - w)) * a.ntx + (c < a.ix0 ? c : c + w);
    }
    return a.iy1 * a.ntx + (i - ntop - nmid);
  }
  return i;
}

template <int K, int V, bool HOT, bool ADJ, bool ACC, bool FULL, int D = 2, bool PHYS = false>
struct Tb2dTile {
  static_assert(V == 4 || V == 8, "V");
  static_assert(!PHYS || (HOT && !ADJ && !ACC) || (!HOT && ADJ), "physical form: forward hotspot or transposed step");
  static_assert(D == 2 || D == 4 || D == 6, "prefetch depth must be even");
  static constexpr int W = 64 * V;    // window width
  static constexpr int RING = tb2d_ring_rows(K);  // hotspot source rows kept in LDS
  static constexpr bool RING_POW2 = (RING & (RING - 1)) == 0;

  const Tb2dArgs& a;
  const int lane;
  int ws, ox0, ox1, y0, y1;
  float S[2][K][V];  // per level: [0] and [1] alternate between "centre" and "oldest/new"
  float Lb[D][V];    // prefetched input rows (D rows in flight)
  float Pb[D][V];    // prefetched power rows
  float Pp[K][V];    // adjoint: running sums carried along the level pipeline
  float cxm[V], cxp[V];
  bool isL[V], isR[V];
  float* ring;       // this wave's LDS ring (HOT forward)
  int slot0;         // ring slot of the current input row

  __device__ __forceinline__ Tb2dTile(const Tb2dArgs& args, int ln, float* lds) : a(args), lane(ln), ring(lds) {}

  template <bool VEC>
  __device__ __forceinline__ void load_row(int r, float (&dstv)[V], const float* base) const {
    const int jr = clampi(r, 0, a.ny - 1);
    const float* rowp = base + (size_t)jr * a.nx;
    const int x0 = ws + lane * V;
    if constexpr (VEC) {
#pragma unroll
      for (int h = 0; h < V; h += 4) {
        const float4 t = *reinterpret_cast<const float4*>(rowp + x0 + h);
        dstv[h] = t.x; dstv[h + 1] = t.y; dstv[h + 2] = t.z; dstv[h + 3] = t.w;
      }
    } else {
#pragma unroll
      for (int v = 0; v < V; ++v) dstv[v] = rowp[clampi(x0 + v, 0, a.nx - 1)];
    }
  }

  template <bool VEC>
  __device__ __forceinline__ void prefetch(int r, int b) {
    load_row<VEC>(r, Lb[b], a.src);
    if constexpr (HOT && !ADJ) load_row<VEC>(r, Pb[b], a.power);
  }

  // Source row of level s (row r+s entered the ring s iterations ago).
  __device__ __forceinline__ void read_q(int s, float (&q)[V]) const {
    if constexpr (HOT && !ADJ) {
      int qs = slot0 - s;
      if constexpr (RING_POW2) qs &= RING - 1;
      else if (qs < 0) qs += RING;
      const float* qp = ring + qs * W + lane * V;
#pragma unroll
      for (int h = 0; h < V; h += 4) {
        const float4 t = *reinterpret_cast<const float4*>(qp + h);
        q[h] = t.x; q[h + 1] = t.y; q[h + 2] = t.z; q[h + 3] = t.w;
      }
    }
  }

  // Phase 1 of a level: source, centre, x-1, x+1 and y+1 terms of row j (oldest row Pr = y+1).
  template <bool XE, bool YE>
  __device__ __forceinline__ void partial(const float (&Pr)[V], const float (&Cr)[V], float (&o)[V], int j,
                                          const float (&q)[V]) const {
    if constexpr (PHYS) {
      // keep the y+1 row (clamped at the last grid row) for phase 2
      const bool botp = YE && (j == a.ny - 1);
#pragma unroll
      for (int v = 0; v < V; ++v) o[v] = botp ? Cr[v] : Pr[v];
      return;
    }
    float wl = 0.0f, eu = 0.0f;
    if constexpr (XE) {
      wl = from_lower(Cr[V - 1]);
      eu = from_upper(Cr[0]);
    }
    const bool bot = YE && (j == a.ny - 1);  // y+1 leaves the grid
    float cyp = a.cf.wy_p;
    if constexpr (ADJ && YE) {
      if (bot) cyp = a.cf.wy_m;
    }
#pragma unroll
    for (int v = 0; v < V; ++v) {
      const float c = Cr[v];
      float xm = (v > 0) ? Cr[v - 1] : wl;
      float xp = (v < V - 1) ? Cr[v + 1] : eu;
      float yp = Pr[v];
      float wxm = a.cf.wx_m, wxp = a.cf.wx_p;
      if constexpr (XE) {
        xm = isL[v] ? c : xm;
        xp = isR[v] ? c : xp;
        wxm = cxm[v];
        wxp = cxp[v];
      }
      if constexpr (YE) yp = bot ? c : yp;
      if constexpr (XE) {
        float acc = centre_term<HOT && !ADJ>(a.cf.c0, c, (HOT && !ADJ) ? q[v] : 0.0f);
        acc = __builtin_fmaf(wxm, xm, acc);
        acc = __builtin_fmaf(wxp, xp, acc);
        acc = __builtin_fmaf(cyp, yp, acc);
        o[v] = acc;
      }
    }
    if constexpr (!XE) {
      // Same term order per cell; the row's two cross-lane terms (x-1 of the first cell, x+1
      // of the last) are issued together behind one DPP hazard wait.
      float acc[V];
#pragma unroll
      for (int v = 0; v < V; ++v) acc[v] = centre_term<HOT && !ADJ>(a.cf.c0, Cr[v], (HOT && !ADJ) ? q[v] : 0.0f);
#pragma unroll
      for (int v = 1; v < V; ++v) acc[v] = __builtin_fmaf(a.cf.wx_m, Cr[v - 1], acc[v]);
      fma_pair_dpp(a.cf.wx_m, Cr[V - 1], acc[0], a.cf.wx_p, Cr[0], acc[V - 1]);
#pragma unroll
      for (int v = 0; v < V - 1; ++v) acc[v] = __builtin_fmaf(a.cf.wx_p, Cr[v + 1], acc[v]);
#pragma unroll
      for (int v = 0; v < V; ++v) o[v] = __builtin_fmaf(cyp, (YE && bot) ? Cr[v] : Pr[v], acc[v]);
    }
  }

  // Phase 2 of a level: add the y-1 term (newest row Nr of the level below).  PHYS: o holds
  // the y+1 row and the whole physical formula is evaluated here, with q the power row.
  template <bool XE, bool YE>
  __device__ __forceinline__ void finish(const float (&Nr)[V], const float (&Cr)[V], float (&o)[V], int j,
                                         const float (&q)[V]) const {
    const bool top = YE && (j == 0);  // y-1 leaves the grid
    if constexpr (PHYS) {
      float sx[V];  // e + w
      if constexpr (XE) {
        const float wl = from_lower(Cr[V - 1]);
        const float eu = from_upper(Cr[0]);
#pragma unroll
        for (int v = 0; v < V; ++v) {
          const float c = Cr[v];
          float xm = (v > 0) ? Cr[v - 1] : wl;
          float xp = (v < V - 1) ? Cr[v + 1] : eu;
          xm = isL[v] ? c : xm;
          xp = isR[v] ? c : xp;
          sx[v] = xp + xm;
        }
      } else {
#pragma unroll
        for (int v = 1; v < V - 1; ++v) sx[v] = Cr[v + 1] + Cr[v - 1];
        add_pair_dpp(Cr[V - 1], Cr[1], sx[0], Cr[0], Cr[V - 2], sx[V - 1]);
      }
#pragma unroll
      for (int v = 0; v < V; ++v) {
        const float c = Cr[v];
        const float yn = (YE && top) ? c : Nr[v];
        // (a + b) - 2c is one rounding of the exact difference: 2c is exact, so it is the
        // fused -2*c + (a + b)
        const float dy = __builtin_fmaf(-2.0f, c, yn + o[v]);
        const float dx = __builtin_fmaf(-2.0f, c, sx[v]);
        const float dz = a.cf.kamb - c;
        float acc = __builtin_fmaf(dy, a.cf.wy_m, (HOT && !ADJ) ? q[v] : 0.0f);
        acc = __builtin_fmaf(dx, a.cf.wx_m, acc);
        acc = __builtin_fmaf(dz, a.cf.wz_m, acc);
        o[v] = __builtin_fmaf(a.cf.cp, acc, c);
      }
      return;
    }
    float cym = a.cf.wy_m;
    if constexpr (ADJ && YE) {
      if (top) cym = a.cf.wy_p;
    }
#pragma unroll
    for (int v = 0; v < V; ++v) {
      float ym = Nr[v];
      if constexpr (YE) ym = top ? Cr[v] : ym;
      o[v] = __builtin_fmaf(cym, ym, o[v]);
    }
  }

  // VEC tiles (nx % 4 == 0, aligned buffers) have window starts, halos, output widths and nx
  // all multiples of 4, so a lane's cells are all inside the output range or all outside it:
  // one predicate and one 16-byte access per lane.
  template <bool XE, bool VEC>
  __device__ __forceinline__ void store_row(int j, const float (&o)[V], float* base) const {
    float* rowp = base + (size_t)j * a.nx;
    const int x0 = ws + lane * V;
    if constexpr (!XE && VEC) {
      if (x0 >= ox0 && x0 < ox1) {
#pragma unroll
        for (int h = 0; h < V; h += 4)
          store4(rowp, x0 + h, a.nx, o[h], o[h + 1], o[h + 2], o[h + 3], a.stream != 0);
      }
    } else {
#pragma unroll
      for (int v = 0; v < V; ++v)
        if (x0 + v >= ox0 && x0 + v < ox1) rowp[x0 + v] = o[v];
    }
  }

  template <bool XE, bool VEC>
  __device__ __forceinline__ void accum_gp(int j, const float (&e)[V]) const {
    float* rowp = a.gp + (size_t)j * a.nx;
    const int x0 = ws + lane * V;
    if constexpr (!XE && VEC) {
      if (x0 >= ox0 && x0 < ox1) {
#pragma unroll
        for (int h = 0; h < V; h += 4) {
          float4* q = reinterpret_cast<float4*>(rowp + x0 + h);
          const float4 g = *q;
          *q = make_float4(__builtin_fmaf(a.cf.cp, e[h], g.x), __builtin_fmaf(a.cf.cp, e[h + 1], g.y),
                           __builtin_fmaf(a.cf.cp, e[h + 2], g.z), __builtin_fmaf(a.cf.cp, e[h + 3], g.w));
        }
      }
    } else {
#pragma unroll
      for (int v = 0; v < V; ++v)
        if (x0 + v >= ox0 && x0 + v < ox1) rowp[x0 + v] = __builtin_fmaf(a.cf.cp, e[v], rowp[x0 + v]);
    }
  }

  // One iteration: input row r arrives (rows stream downwards in index), level s makes row r+s.
  // LB is the prefetch slot of row r (the loop is unrolled by D, a multiple of the state period 2).
  template <int LB, bool XE, bool YE, bool VEC>
  __device__ __forceinline__ void step(int r) {
    constexpr int ROT = LB & 1;
    float (&X)[K][V] = S[ROT];      // oldest rows on entry; partial sums; newest rows on exit
    float (&C)[K][V] = S[ROT ^ 1];  // centre rows
    const int keff = FULL ? K : a.keff;
    // ---- phase 1, top level first: partial[s] (row r+s) replaces X[s] once X[s] is used
    float part_top[V];
    // source rows are read one level ahead so that only two of them are live at a time
    float qc[V], qn[V];
    (void)qc;
    (void)qn;
    if constexpr (!PHYS) read_q(K, qc);
#pragma unroll
    for (int s = K; s >= 1; --s) {
      const int j = r + s;
      if constexpr (HOT && !ADJ && !PHYS) {
        if (s > 1) read_q(s - 1, qn);
      }
      float o[V];
      if (FULL || s <= keff) {
        partial<XE, YE>(X[s - 1], C[s - 1], o, j, qc);
      } else {
#pragma unroll
        for (int v = 0; v < V; ++v) o[v] = 0.0f;  // surplus level: overwritten in phase 2
      }
#pragma unroll
      for (int v = 0; v < V; ++v) {
        if (s == K) part_top[v] = o[v];
        else X[s][v] = o[v];
      }
      if constexpr (HOT && !ADJ && !PHYS) {
#pragma unroll
        for (int v = 0; v < V; ++v) qc[v] = qn[v];
      }
    }
    // ---- phase 2, bottom level first
#pragma unroll
    for (int v = 0; v < V; ++v) X[0][v] = Lb[LB][v];
    if constexpr (HOT && !ADJ) {
      float* qp = ring + slot0 * W + lane * V;
      if constexpr (PHYS) {
#pragma unroll
        for (int v = 0; v < V; ++v) qp[v] = Pb[LB][v];
      } else {
#pragma unroll
        for (int v = 0; v < V; ++v) qp[v] = __builtin_fmaf(a.cf.cp, Pb[LB][v], a.cf.kamb);
      }
    }
    prefetch<VEC>(r - D, LB);
    float Pn[K][V];
    (void)Pn;
#pragma unroll
    for (int s = 1; s <= K; ++s) {
      const int j = r + s;
      float o[V];
#pragma unroll
      for (int v = 0; v < V; ++v) o[v] = (s == K) ? part_top[v] : X[s][v];
      if (FULL || s <= keff) {
        float qv[V];
        if constexpr (PHYS) read_q(s, qv);
        finish<XE, YE>(X[s - 1], C[s - 1], o, j, qv);
      } else {
#pragma unroll
        for (int v = 0; v < V; ++v) o[v] = C[s - 1][v];  // surplus level: forward its input row
      }
      if constexpr (ACC) {
        if (s < K) {
          const bool add = FULL ? true : (s < keff);
#pragma unroll
          for (int v = 0; v < V; ++v) {
            const float prev = (s == 1) ? C[0][v] : Pp[s - 1][v];
            Pn[s][v] = add ? prev + o[v] : prev;
          }
        }
      }
      if (s < K) {
#pragma unroll
        for (int v = 0; v < V; ++v) X[s][v] = o[v];
      } else if (j >= y0 && j < y1) {
        store_row<XE, VEC>(j, o, a.dst);
        if constexpr (ACC) {
          float e[V];
#pragma unroll
          for (int v = 0; v < V; ++v) e[v] = (K == 1) ? C[0][v] : Pp[K - 1][v];
          accum_gp<XE, VEC>(j, e);
        }
      }
    }
    if constexpr (ACC) {
#pragma unroll
      for (int s = 1; s < K; ++s)
#pragma unroll
        for (int v = 0; v < V; ++v) Pp[s][v] = Pn[s][v];
    }
    if constexpr (HOT && !ADJ) {
      if constexpr (RING_POW2) slot0 = (slot0 + 1) & (RING - 1);
      else slot0 = (slot0 + 1 == RING) ? 0 : slot0 + 1;
    }
  }

  template <bool XE, bool YE, bool VEC>
  __device__ __forceinline__ void run() {
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int s = 0; s < K; ++s)
#pragma unroll
        for (int v = 0; v < V; ++v) S[b][s][v] = 0.0f;
    if constexpr (ACC) {
#pragma unroll
      for (int s = 0; s < K; ++s)
#pragma unroll
        for (int v = 0; v < V; ++v) Pp[s][v] = 0.0f;
    }
    const int keff = FULL ? K : a.keff;
    // input rows from y1-1+keff down to y0-keff; level K emits row r+K
    const int r0 = y1 - 1 + keff;
    int nit = (y1 - y0) + keff + K;
    nit = (nit + D - 1) / D * D;  // the extra iterations only touch rows outside [y0, y1)
    slot0 = 0;
#pragma unroll
    for (int b = 0; b < D; ++b) prefetch<VEC>(r0 - b, b);
    for (int it = 0; it < nit; it += D) {
      step<0, XE, YE, VEC>(r0 - it);
      step<1, XE, YE, VEC>(r0 - it - 1);
      if constexpr (D >= 4) {
        step<2 % D, XE, YE, VEC>(r0 - it - 2);
        step<3 % D, XE, YE, VEC>(r0 - it - 3);
      }
      if constexpr (D >= 6) {
        step<4 % D, XE, YE, VEC>(r0 - it - 4);
        step<5 % D, XE, YE, VEC>(r0 - it - 5);
      }
    }
  }

  // INTERIOR: the tile is known to touch no grid edge and the buffers to be aligned, so only
  // the edge-free body is compiled in (fewer registers than the kernel with every variant).
  template <bool INTERIOR = false>
  __device__ __forceinline__ void process(int tile) {
    const int tx = tile % a.ntx;
    const int sg = tile / a.ntx;
    ox0 = tx * a.cs;
    ox1 = min(ox0 + a.cs, a.nx);
    ws = ox0 - a.kr;
    y0 = a.ylo + sg * a.seg;
    y1 = min(y0 + a.seg, a.yhi);
    const bool xe = (ws < 0) || (ws + W > a.nx);
    const int keff = FULL ? K : a.keff;
    const bool ye = (y0 - keff <= 0) || (y1 + keff >= a.ny);
#pragma unroll
    for (int v = 0; v < V; ++v) {
      const int x = ws + lane * V + v;
      isL[v] = (x == 0);
      isR[v] = (x == a.nx - 1);
      cxm[v] = a.cf.wx_m;
      cxp[v] = a.cf.wx_p;
      if constexpr (ADJ) {
        if (isL[v]) cxm[v] = a.cf.wx_p;
        if (isR[v]) cxp[v] = a.cf.wx_m;
      }
    }
    if constexpr (INTERIOR) {
      run<false, false, true>();
    } else {
      if (xe) {
        if (ye) run<true, true, false>(); else run<true, false, false>();
      } else if (a.aligned) {
        if (ye) run<false, true, true>(); else run<false, false, true>();
      } else {
        if (ye) run<false, true, false>(); else run<false, false, false>();
      }
    }
  }
};

// One workgroup (one wave) per tile of the launch's part (gridDim.x tiles).  INTERIOR = true
// is the kernel for part 1; part 0 and part 2 use INTERIOR = false.
template <int K, int V, bool HOT, bool ADJ, bool ACC, bool FULL, int D, bool INTERIOR, bool PHYS = false>
__global__ __launch_bounds__(64) void tb2d_kernel(Tb2dArgs a) {
  constexpr int RING = (HOT && !ADJ) ? tb2d_ring_rows(K) : 1;
  __shared__ __align__(16) float ring[RING * 64 * V];
  const int tile = tb2d_part_tile(a, xcd_remap(blockIdx.x, gridDim.x));
  Tb2dTile<K, V, HOT, ADJ, ACC, FULL, D, PHYS> t(a, threadIdx.x, ring);
  t.template process<INTERIOR>(tile);
}

// Tiles in the launch of part a.part.
inline int tb2d_part_tiles(const Tb2dArgs& a) {
  const int interior = (a.ix1 - a.ix0) * (a.iy1 - a.iy0);
  if (a.part == 1) return interior;
  if (a.part == 2) return a.ntx * a.nseg - interior;
  return a.ntx * a.nseg;
}

// Launch shape of the 2D kernels: 256-column windows (one wave, 4 cells per lane), one
// workgroup per (x tile, row segment).
constexpr int kTb2dV = 4;
// Rows in flight per wave: four for diffusion; two where the hotspot source ring or the
// adjoint's running sums already take the registers, except in the edge-free hotspot kernel
// for 8 < K <= 12, which has the registers for four (168 VGPRs) within the occupancy its
// 16 KiB ring allows (+7%).
#define TB2D_DEPTH(K, HOT, ADJ, INTERIOR) \
  ((!(HOT) && !(ADJ)) ? 4 : ((HOT) && !(ADJ) && (INTERIOR) && (K) > 8 && (K) <= 12) ? 4 : 2)
#define TB_LAUNCH2D_F(K, HOT, ADJ, ACC, FULL, PHYS, a, s)                                               \
  do {                                                                                                  \
    if ((a).part == 1)                                                                                  \
      hipLaunchKernelGGL((tb2d_kernel<K, kTb2dV, HOT, ADJ, ACC, FULL, TB2D_DEPTH(K, HOT, ADJ, true), true, PHYS>), \
                         dim3(tb2d_part_tiles(a)), dim3(64), 0, s, a);                                  \
    else                                                                                                \
      hipLaunchKernelGGL((tb2d_kernel<K, kTb2dV, HOT, ADJ, ACC, FULL, TB2D_DEPTH(K, HOT, ADJ, false), false, PHYS>), \
                         dim3(tb2d_part_tiles(a)), dim3(64), 0, s, a);                                  \
    return hipGetLastError();                                                                           \
  } while (0)
#define TB_LAUNCH2D(K, HOT, ADJ, ACC, FULL, a, s) TB_LAUNCH2D_F(K, HOT, ADJ, ACC, FULL, false, a, s)
