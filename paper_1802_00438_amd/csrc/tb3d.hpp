// tb3d.hpp -- temporal-blocked 3D star stencil: x-y tiles streamed along z ("2.5D").
//
// Method (paper Sections 3.1, 3.2; Eq. 2, 4, 5): 2D spatial blocking in x and y with
// overlapping halos of k cells, streaming (no blocking) along z, and k consecutive time steps
// applied to a block before it returns to memory; step s trails step s-1 by one plane.
//
// gfx950 mapping:
//   * A workgroup of NW wavefronts owns a window of (64*V) x (R*NW) cells in x-y.  Lane l
//     of wave w holds the V x R patch x in [xw + l*V, +V), y in [yw + w*R, +R) of every plane,
//     so each row of a plane is one coalesced 8-byte access per lane.
//   * Planes stream upwards in z.  Level s (1..K) computes plane r-s while level 0 receives
//     plane r.  The canonical term order (centre, x-1, x+1, y+1, y-1, z-1, z+1) ends with the
//     plane that arrived first (z-1) followed by the plane that arrives last (z+1), so each
//     iteration runs in two phases: (1) for every level, fold the centre plane (with its
//     in-plane neighbours) and the oldest plane into a partial sum, freeing the oldest
//     plane's registers; (2) walking up the levels, add the z+1 term from the plane the level
//     below has just produced.  Each level keeps two planes in registers (the register
//     analogue of the paper's 3D shift register, Eq. 1); the plane loop, unrolled by two,
//     renames them without copies.
//   * In-plane neighbours: x across lanes by DPP wave shifts, y inside a lane's R rows
//     directly, and y across waves through LDS: every new level plane publishes its first
//     and last rows, and one barrier per plane (double-buffered by plane parity) makes them
//     visible to the next plane's phase 1, for all k levels at once.  In a window flush with
//     a y edge of the grid, the outermost wave reads its own edge row there instead.
//   * Clamp-to-edge is applied per level by using the cell's own value for an out-of-grid
//     neighbour; tiles that touch no x/y edge run code with no boundary handling, and the z
//     edges cost only on the few planes that meet them.
//   * Hotspot: in a pass of all K steps the source q = fma(cp, p, kamb) of a plane is formed
//     once, when it becomes the newest output plane (level 1), from a power plane loaded an
//     iteration ahead; levels 2..K read it back from an LDS ring of K-1 planes that holds each
//     lane's own cells.  A shorter pass re-forms it per level from the power plane.
//   * Adjoint: transposed operator (mirrored weights, zero outside the grid, self term with
//     the weight of the leaving direction); sum_s lambda_s travels with the pipeline and is
//     added to grad_p once per pass.
#pragma once
#include "device_common.hpp"

struct Tb3dArgs {
  const float* src;
  float* dst;
  const float* power;  // forward hotspot
  float* gp;           // adjoint hotspot accumulator or null
  int nx, ny, nz;
  int keff;
  int csx, csy;        // output cells per tile in x and y
  int krx, kry;        // window offsets (window start = tile start - kr)
  int ntx, nty;        // tiles in x, y
  int segz, nsegz;     // output planes per tile, tiles along z
  int nwork;           // > 0: balanced launch of nwork workgroups (see tb3d_kernel)
  // Edge-flush tiling (forward kernels, grids at least one window wide/high): the first and
  // last tile of an axis place their window flush with the grid edge and output fx (fy)
  // cells from it; the tiles between output csx (csy) cells each.  0: uniform tiling.
  // ax = 2: a grid narrower than a window with nx even: one window per row of tiles, flush
  // with x = 0, its lanes past the row idle.
  int ax, ay, fx, fy;
  int aligned;         // 1: nx even and 8-byte aligned buffers (vector access in interior tiles)
  // Output planes [zlo, zhi); tiles (and balanced shares) cover only them.  Every plane
  // normally; a slab pass with ghost planes stores only the planes between them.
  int zlo, zhi;
  DevCoef cf;
};

template <int K, int V, int R, int NW, bool HOT, bool ADJ, bool ACC, bool FULL, int PD = 1>
struct Tb3dTile {
  static constexpr int WX = 64 * V;
  static constexpr int WY = R * NW;
  const Tb3dArgs& a;
  const int lane, wave;
  int xw, yw, ox0, ox1, oy0, oy1, z0, z1;
  float S[2][K][R][V];  // per level: centre plane and oldest/partial/newest plane, alternating
  float Lb[PD][R][V];   // next PD input planes (loaded PD iterations ahead)
  float Qb[R][V];       // hotspot: the power plane of the next iteration's newest output plane
  float Pp[K][R][V];
  float cxm[V], cxp[V];
  bool isL[V], isR[V];
  bool rowTop[R], rowBot[R];  // wave-uniform: strip row is grid row 0 / ny-1
  bool topA, botA;            // window flush with grid row 0 / ny-1 (edge-flush tiling)
  bool pastR;                 // narrow window (a.ax == 2): this lane holds x = nx
  // LDS sources of this wave's halo rows, as offsets within one level's block of hal: the
  // last row of the wave above (y-1) and the first row of the wave below (y+1).  The outermost
  // wave of a window flush with row 0 (ny-1) takes its own first (last) row instead, which is
  // exactly the clamp, at no cost per cell.
  int hn_off, hs_off;
  float* hal;                 // LDS: [2][K][NW][2][WX]
  // Hotspot forward: q = fma(cp, p, kamb) of the K-1 planes before the newest output plane,
  // one slot per plane (plane j in slot j mod (K-1)), each lane's own cells only:
  // [K-1][NW][R][64][V].
  static constexpr bool QONCE = HOT && !ADJ && FULL;  // passes of all K steps
  static constexpr int QR = (QONCE && K > 1) ? K - 1 : 0;
  float* qring;

  __device__ __forceinline__ Tb3dTile(const Tb3dArgs& args, int ln, int wv, float* lds, float* qlds = nullptr)
      : a(args), lane(ln), wave(wv), hal(lds), qring(qlds) {}

  __device__ __forceinline__ float* qslot(int plane, int r) const {
    int sl = plane % QR;
    if (sl < 0) sl += QR;
    return qring + (((sl * NW + wave) * R + r) * 64 + lane) * V;
  }

  __device__ __forceinline__ float* hrow(int buf, int lev, int w, int which) const {
    return hal + ((((buf * K + lev) * NW + w) * 2 + which) * WX);
  }

  // EA == 2 (a window wider than the grid): lanes past the row load its last two cells
  // instead, so every access stays inside the row.
  template <bool XE, int EA = 0>
  __device__ __forceinline__ void load_plane(int z, float (&d)[R][V], const float* base) const {
    const int zc = clampi(z, 0, a.nz - 1);
    const float* pl = base + (size_t)zc * a.ny * a.nx;
    const int x0 = (EA == 2) ? min(xw + lane * V, a.nx - V) : xw + lane * V;
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int y = clampi(yw + wave * R + r, 0, a.ny - 1);
      const float* rowp = pl + (size_t)y * a.nx;
      if constexpr (!XE && V == 2) {
        const float2 t = *reinterpret_cast<const float2*>(rowp + x0);
        d[r][0] = t.x; d[r][1] = t.y;
      } else {
#pragma unroll
        for (int v = 0; v < V; ++v) d[r][v] = rowp[XE ? clampi(x0 + v, 0, a.nx - 1) : x0 + v];
      }
    }
  }

  __device__ __forceinline__ void publish(int buf, int lev, const float (&pl)[R][V]) const {
    float* t = hrow(buf, lev, wave, 0) + lane * V;
    float* b = hrow(buf, lev, wave, 1) + lane * V;
#pragma unroll
    for (int v = 0; v < V; ++v) {
      t[v] = pl[0][v];
      b[v] = pl[R - 1][v];
    }
  }

  // Phase 1: source, in-plane terms of centre plane Cl (cross-wave rows from LDS buffer rbuf)
  // and the z-1 term of the oldest plane Pl, for output plane j.
  // XE/YE: generic clamping of every cell (windows that cross a grid edge).  EA: window flush
  // with an x edge of the grid (edge-flush tiling): an end lane that holds x = 0 or x = nx-1
  // keeps its own value in the cross-lane move, which is exactly the clamp.  A window flush
  // with row 0 or ny-1 needs nothing here: its outermost wave reads its own edge row as the
  // halo row (hn_off, hs_off).  The transposed step also takes EA for y-flush windows, where
  // the flush rows swap the weight of the leaving direction.
  template <bool XE, bool YE, bool ZE, int EA>
  __device__ __forceinline__ void partial(const float (&Pl)[R][V], const float (&Cl)[R][V], float (&o)[R][V],
                                          int lev_in, int rbuf, int j, const float (&qin)[R][V]) const {
    float q[R][V];
    (void)q;
    (void)qin;
    if constexpr (QONCE) {
#pragma unroll
      for (int r = 0; r < R; ++r)
#pragma unroll
        for (int v = 0; v < V; ++v) q[r][v] = qin[r][v];
    } else if constexpr (HOT && !ADJ) {
      // passes of fewer than K steps re-form the source per level (the ring's registers
      // would spill there)
      const int zc = clampi(j, 0, a.nz - 1);
      const float* pl = a.power + (size_t)zc * a.ny * a.nx;
      const int x0 = (EA == 2) ? min(xw + lane * V, a.nx - V) : xw + lane * V;
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const int y = clampi(yw + wave * R + r, 0, a.ny - 1);
        const float* rowp = pl + (size_t)y * a.nx;
        if constexpr (!XE && V == 2) {
          const float2 t = *reinterpret_cast<const float2*>(rowp + x0);
          q[r][0] = __builtin_fmaf(a.cf.cp, t.x, a.cf.kamb);
          q[r][1] = __builtin_fmaf(a.cf.cp, t.y, a.cf.kamb);
        } else {
#pragma unroll
          for (int v = 0; v < V; ++v)
            q[r][v] = __builtin_fmaf(a.cf.cp, rowp[XE ? clampi(x0 + v, 0, a.nx - 1) : x0 + v], a.cf.kamb);
        }
      }
    }
    float hn[V], hs[V];
    {
      const float* lev = hrow(rbuf, lev_in, 0, 0) + lane * V;
      const float* pn = lev + hn_off;
      const float* ps = lev + hs_off;
#pragma unroll
      for (int v = 0; v < V; ++v) {
        hn[v] = pn[v];
        hs[v] = ps[v];
      }
    }
    const bool zlo = ZE && (j == 0);
    float czm = a.cf.wz_m;
    if constexpr (ADJ && ZE) {
      if (zlo) czm = a.cf.wz_p;
    }
#pragma unroll
    for (int r = 0; r < R; ++r) {
      float wl = 0.0f, eu = 0.0f;
      if constexpr (XE) {
        wl = from_lower(Cl[r][V - 1]);
        eu = from_upper(Cl[r][0]);
      } else if constexpr (EA == 2) {
        // window wider than the grid: lane 0 keeps its own value as in a flush window; the
        // lane that holds x = nx passes on its left neighbour's last cell, so cell nx - 1
        // reads its own value as its x+1 neighbour, which is the clamp
        wl = from_lower_or(Cl[r][V - 1], Cl[r][0]);
        eu = from_upper(pastR ? wl : Cl[r][0]);
      } else if constexpr (EA) {
        wl = from_lower_or(Cl[r][V - 1], Cl[r][0]);
        eu = from_upper_or(Cl[r][0], Cl[r][V - 1]);
      }
      float cym = a.cf.wy_m, cyp = a.cf.wy_p;
      if constexpr (ADJ && YE) {
        if (rowTop[r]) cym = a.cf.wy_p;
        if (rowBot[r]) cyp = a.cf.wy_m;
      }
      if constexpr (ADJ && EA && !YE) {
        // transposed step at a flush edge row: the leaving direction's weight on the own value
        if (r == 0 && topA && wave == 0) cym = a.cf.wy_p;
        if (r == R - 1 && botA && wave == NW - 1) cyp = a.cf.wy_m;
      }
#pragma unroll
      for (int v = 0; v < V; ++v) {
        const float c = Cl[r][v];
        float xm = (v > 0) ? Cl[r][v - 1] : wl;
        float xp = (v < V - 1) ? Cl[r][v + 1] : eu;
        float ym = (r > 0) ? Cl[r - 1][v] : hn[v];
        float yp = (r < R - 1) ? Cl[r + 1][v] : hs[v];
        float zm = Pl[r][v];
        float wxm = a.cf.wx_m, wxp = a.cf.wx_p;
        if constexpr (XE) {
          xm = isL[v] ? c : xm;
          xp = isR[v] ? c : xp;
          wxm = cxm[v];
          wxp = cxp[v];
        } else if constexpr (EA && ADJ) {
          wxm = cxm[v];  // per-lane weights: the leaving direction's weight at x = 0 / nx-1
          wxp = cxp[v];
        }
        if constexpr (YE) {
          ym = rowTop[r] ? c : ym;
          yp = rowBot[r] ? c : yp;
        }
        if constexpr (ZE) zm = zlo ? c : zm;
        if constexpr (XE || EA) {
          float acc =
              upd2<HOT && !ADJ>(a.cf.c0, c, wxm, xm, wxp, xp, cyp, yp, cym, ym, (HOT && !ADJ) ? q[r][v] : 0.0f);
          o[r][v] = __builtin_fmaf(czm, zm, acc);
        }
      }
      if constexpr (!XE && !EA) {
        // Same term order per cell; the row's two cross-lane terms (x-1 of the first cell,
        // x+1 of the last) are issued together behind one DPP hazard wait.
        float acc[V];
#pragma unroll
        for (int v = 0; v < V; ++v)
          acc[v] = centre_term<HOT && !ADJ>(a.cf.c0, Cl[r][v], (HOT && !ADJ) ? q[r][v] : 0.0f);
#pragma unroll
        for (int v = 1; v < V; ++v) acc[v] = __builtin_fmaf(a.cf.wx_m, Cl[r][v - 1], acc[v]);
        fma_pair_dpp(a.cf.wx_m, Cl[r][V - 1], acc[0], a.cf.wx_p, Cl[r][0], acc[V - 1]);
#pragma unroll
        for (int v = 0; v < V - 1; ++v) acc[v] = __builtin_fmaf(a.cf.wx_p, Cl[r][v + 1], acc[v]);
#pragma unroll
        for (int v = 0; v < V; ++v) {
          const float c = Cl[r][v];
          float ym = (r > 0) ? Cl[r - 1][v] : hn[v];
          float yp = (r < R - 1) ? Cl[r + 1][v] : hs[v];
          float zm = Pl[r][v];
          if constexpr (YE) {
            ym = rowTop[r] ? c : ym;
            yp = rowBot[r] ? c : yp;
          }
          if constexpr (ZE) zm = zlo ? c : zm;
          float t = __builtin_fmaf(cyp, yp, acc[v]);
          t = __builtin_fmaf(cym, ym, t);
          o[r][v] = __builtin_fmaf(czm, zm, t);
        }
      }
    }
  }

  // Phase 2: z+1 term from the newest plane Nl of the level below.
  template <bool ZE>
  __device__ __forceinline__ void finish(const float (&Nl)[R][V], const float (&Cl)[R][V], float (&o)[R][V],
                                         int j) const {
    const bool zhi = ZE && (j == a.nz - 1);
    float czp = a.cf.wz_p;
    if constexpr (ADJ && ZE) {
      if (zhi) czp = a.cf.wz_m;
    }
#pragma unroll
    for (int r = 0; r < R; ++r)
#pragma unroll
      for (int v = 0; v < V; ++v) {
        float zp = Nl[r][v];
        if constexpr (ZE) zp = zhi ? Cl[r][v] : zp;
        o[r][v] = __builtin_fmaf(czp, zp, o[r][v]);
      }
  }

  template <bool XE>
  __device__ __forceinline__ void store_plane(int j, const float (&o)[R][V]) const {
    float* pl = a.dst + (size_t)j * a.ny * a.nx;
    const int x0 = xw + lane * V;
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int y = yw + wave * R + r;
      if (y < oy0 || y >= oy1) continue;
      float* rowp = pl + (size_t)y * a.nx;
      if constexpr (!XE && V == 2) {
        // edge-free tiles: window starts and output bounds are all even (nx even), so a lane's
        // two cells are both inside the output range or both outside it
        if (x0 >= ox0 && x0 < ox1) *reinterpret_cast<float2*>(rowp + x0) = make_float2(o[r][0], o[r][1]);
      } else {
#pragma unroll
        for (int v = 0; v < V; ++v)
          if (x0 + v >= ox0 && x0 + v < ox1) rowp[x0 + v] = o[r][v];
      }
    }
  }

  template <bool XE>
  __device__ __forceinline__ void accum_gp(int j, const float (&e)[R][V]) const {
    float* pl = a.gp + (size_t)j * a.ny * a.nx;
    const int x0 = xw + lane * V;
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int y = yw + wave * R + r;
      if (y < oy0 || y >= oy1) continue;
      float* rowp = pl + (size_t)y * a.nx;
      if constexpr (!XE && V == 2) {
        if (x0 >= ox0 && x0 < ox1) {
          float2* q = reinterpret_cast<float2*>(rowp + x0);
          const float2 g = *q;
          *q = make_float2(__builtin_fmaf(a.cf.cp, e[r][0], g.x), __builtin_fmaf(a.cf.cp, e[r][1], g.y));
        }
      } else {
#pragma unroll
        for (int v = 0; v < V; ++v)
          if (x0 + v >= ox0 && x0 + v < ox1) rowp[x0 + v] = __builtin_fmaf(a.cf.cp, e[r][v], rowp[x0 + v]);
      }
    }
  }

  // Iteration with input plane r: level s computes plane r - s.  Planes made in this
  // iteration publish their edge rows in LDS buffer ROT; phase 1 reads the centre planes'
  // edge rows published in the previous iteration (buffer ROT ^ 1).
  template <int ROT, bool XE, bool YE, bool ZE, int EA>
  __device__ __forceinline__ void step(int r) {
    float (&X)[K][R][V] = S[ROT];      // oldest planes on entry, partial sums, newest on exit
    float (&C)[K][R][V] = S[ROT ^ 1];  // centre planes
    const int keff = FULL ? K : a.keff;
    float part_top[R][V];
#pragma unroll
    for (int s = K; s >= 1; --s) {
      const int j = r - s;
      float o[R][V];
      float q[R][V];
      (void)q;
      if constexpr (QONCE) {
        if (s == 1) {
          // the newest output plane's source, from the power plane loaded an iteration ahead;
          // the older planes' sources come from the ring, where this one goes for them
#pragma unroll
          for (int rr = 0; rr < R; ++rr)
#pragma unroll
            for (int v = 0; v < V; ++v) q[rr][v] = __builtin_fmaf(a.cf.cp, Qb[rr][v], a.cf.kamb);
          if constexpr (QR > 0) {
#pragma unroll
            for (int rr = 0; rr < R; ++rr) {
              float* d = qslot(j, rr);
#pragma unroll
              for (int v = 0; v < V; ++v) d[v] = q[rr][v];
            }
          }
        } else {
#pragma unroll
          for (int rr = 0; rr < R; ++rr) {
            const float* d = qslot(j, rr);
#pragma unroll
            for (int v = 0; v < V; ++v) q[rr][v] = d[v];
          }
        }
      }
      if (FULL || s <= keff) {
        partial<XE, YE, ZE, EA>(X[s - 1], C[s - 1], o, s - 1, ROT ^ 1, j, q);
      } else {
#pragma unroll
        for (int rr = 0; rr < R; ++rr)
#pragma unroll
          for (int v = 0; v < V; ++v) o[rr][v] = 0.0f;
      }
#pragma unroll
      for (int rr = 0; rr < R; ++rr)
#pragma unroll
        for (int v = 0; v < V; ++v) {
          if (s == K) part_top[rr][v] = o[rr][v];
          else X[s][rr][v] = o[rr][v];
        }
    }
    constexpr int LB = ROT % PD;  // plane r arrived in Lb[LB]; plane r + PD replaces it
#pragma unroll
    for (int rr = 0; rr < R; ++rr)
#pragma unroll
      for (int v = 0; v < V; ++v) X[0][rr][v] = Lb[LB][rr][v];
    load_plane<XE, EA>(r + PD, Lb[LB], a.src);
    if constexpr (QONCE) load_plane<XE, EA>(r, Qb, a.power);  // for plane r, the next newest
    publish(ROT, 0, X[0]);
    float Pn[K][R][V];
    (void)Pn;
#pragma unroll
    for (int s = 1; s <= K; ++s) {
      const int j = r - s;
      float o[R][V];
#pragma unroll
      for (int rr = 0; rr < R; ++rr)
#pragma unroll
        for (int v = 0; v < V; ++v) o[rr][v] = (s == K) ? part_top[rr][v] : X[s][rr][v];
      if (FULL || s <= keff) {
        finish<ZE>(X[s - 1], C[s - 1], o, j);
      } else {
#pragma unroll
        for (int rr = 0; rr < R; ++rr)
#pragma unroll
          for (int v = 0; v < V; ++v) o[rr][v] = C[s - 1][rr][v];
      }
      if constexpr (ACC) {
        if (s < K) {
          const bool add = FULL ? true : (s < keff);
#pragma unroll
          for (int rr = 0; rr < R; ++rr)
#pragma unroll
            for (int v = 0; v < V; ++v) {
              const float prev = (s == 1) ? C[0][rr][v] : Pp[s - 1][rr][v];
              Pn[s][rr][v] = add ? prev + o[rr][v] : prev;
            }
        }
      }
      if (s < K) {
#pragma unroll
        for (int rr = 0; rr < R; ++rr)
#pragma unroll
          for (int v = 0; v < V; ++v) X[s][rr][v] = o[rr][v];
        publish(ROT, s, o);
      } else if (j >= z0 && j < z1) {
        store_plane<XE>(j, o);
        if constexpr (ACC) {
          float e[R][V];
#pragma unroll
          for (int rr = 0; rr < R; ++rr)
#pragma unroll
            for (int v = 0; v < V; ++v) e[rr][v] = (K == 1) ? C[0][rr][v] : Pp[K - 1][rr][v];
          accum_gp<XE>(j, e);
        }
      }
    }
    if constexpr (ACC) {
#pragma unroll
      for (int s = 1; s < K; ++s)
#pragma unroll
        for (int rr = 0; rr < R; ++rr)
#pragma unroll
          for (int v = 0; v < V; ++v) Pp[s][rr][v] = Pn[s][rr][v];
    }
    __syncthreads();
  }

  template <bool XE, bool YE, int EA>
  __device__ __forceinline__ void run() {
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int s = 0; s < K; ++s)
#pragma unroll
        for (int rr = 0; rr < R; ++rr)
#pragma unroll
          for (int v = 0; v < V; ++v) S[b][s][rr][v] = 0.0f;
    if constexpr (ACC) {
#pragma unroll
      for (int s = 0; s < K; ++s)
#pragma unroll
        for (int rr = 0; rr < R; ++rr)
#pragma unroll
          for (int v = 0; v < V; ++v) Pp[s][rr][v] = 0.0f;
    }
    const int keff = FULL ? K : a.keff;
    const int r0 = z0 - keff;
    int nit = (z1 - z0) + keff + K;
    nit = (nit + 1) & ~1;
#pragma unroll
    for (int d = 0; d < PD; ++d) load_plane<XE, EA>(r0 + d, Lb[d], a.src);
    if constexpr (QONCE) load_plane<XE, EA>(r0 - 1, Qb, a.power);
    // Pairs of iterations that compute a plane at a z edge form a prefix (z = 0) and a suffix
    // (z = nz-1) of the loop; they run a body with z-edge handling, the rest a body without
    // it.  Separate loops (rather than a branch inside one loop) keep the register allocation
    // of the hot body free of merge copies.
    int it = 0;
    auto edge = [&](int i) {
      const int r = r0 + i;
      return (r - K <= 0 && r >= 0) || (r - K <= a.nz - 1 && r >= a.nz - 1);
    };
    for (; it < nit && edge(it); it += 2) {
      step<0, XE, YE, true, EA>(r0 + it);
      step<1, XE, YE, true, EA>(r0 + it + 1);
    }
    for (; it < nit && !edge(it); it += 2) {
      step<0, XE, YE, false, EA>(r0 + it);
      step<1, XE, YE, false, EA>(r0 + it + 1);
    }
    for (; it < nit; it += 2) {
      step<0, XE, YE, true, EA>(r0 + it);
      step<1, XE, YE, true, EA>(r0 + it + 1);
    }
  }

  // Tile `tile` of the (x, y, z-segment) tiling.
  __device__ __forceinline__ void process(int tile) {
    const int tx = tile % a.ntx;
    const int rest = tile / a.ntx;
    const int ty = rest % a.nty;
    const int tz = rest / a.nty;
    process_column(tx, ty, a.zlo + tz * a.segz, min(a.zlo + tz * a.segz + a.segz, a.zhi));
  }

  // Output planes [zs, ze) of the x-y column (tx, ty).
  __device__ __forceinline__ void process_column(int tx, int ty, int zs, int ze) {
    if (a.ax == 2) {
      ox0 = 0; ox1 = a.nx; xw = 0;  // one window, flush with x = 0, wider than the grid
    } else if (a.ax) {
      if (a.ntx == 1) { ox0 = 0; ox1 = a.nx; xw = 0; }
      else if (tx == 0) { ox0 = 0; ox1 = a.fx; xw = 0; }
      else if (tx == a.ntx - 1) { ox0 = max(a.fx, a.nx - a.fx); ox1 = a.nx; xw = a.nx - WX; }
      else { ox0 = a.fx + (tx - 1) * a.csx; ox1 = min(ox0 + a.csx, a.nx - a.fx); xw = ox0 - a.krx; }
    } else {
      ox0 = tx * a.csx;
      ox1 = min(ox0 + a.csx, a.nx);
      xw = ox0 - a.krx;
    }
    if (a.ay) {
      if (a.nty == 1) { oy0 = 0; oy1 = a.ny; yw = 0; }
      else if (ty == 0) { oy0 = 0; oy1 = a.fy; yw = 0; }
      else if (ty == a.nty - 1) { oy0 = max(a.fy, a.ny - a.fy); oy1 = a.ny; yw = a.ny - WY; }
      else { oy0 = a.fy + (ty - 1) * a.csy; oy1 = min(oy0 + a.csy, a.ny - a.fy); yw = oy0 - a.kry; }
    } else {
      oy0 = ty * a.csy;
      oy1 = min(oy0 + a.csy, a.ny);
      yw = oy0 - a.kry;
    }
    const bool xa = a.ax && (tx == 0 || tx == a.ntx - 1);
    topA = a.ay && ty == 0;
    botA = a.ay && ty == a.nty - 1;
    {
      const int wn = (wave == 0) ? 0 : wave - 1, which_n = (wave == 0 && topA) ? 0 : 1;
      const int ws_ = (wave == NW - 1) ? NW - 1 : wave + 1, which_s = (wave == NW - 1 && botA) ? 1 : 0;
      hn_off = (wn * 2 + which_n) * WX;
      hs_off = (ws_ * 2 + which_s) * WX;
    }
    z0 = zs;
    z1 = ze;
    const bool xe = !a.aligned || (xw < 0) || (xw + WX > a.nx && a.ax != 2);
    pastR = (xw + lane * V == a.nx);
    const bool ye = (yw < 0) || (yw + WY > a.ny);
#pragma unroll
    for (int v = 0; v < V; ++v) {
      const int x = xw + lane * V + v;
      isL[v] = (x == 0);
      isR[v] = (x == a.nx - 1);
      cxm[v] = a.cf.wx_m;
      cxp[v] = a.cf.wx_p;
      if constexpr (ADJ) {
        if (isL[v]) cxm[v] = a.cf.wx_p;
        if (isR[v]) cxp[v] = a.cf.wx_m;
      }
    }
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int y = yw + wave * R + r;
      rowTop[r] = (y == 0);
      rowBot[r] = (y == a.ny - 1);
    }
    // A window that needs generic clamping on one axis takes the generic body on the other
    // axis too when that axis has a flush window (the generic bodies clamp any placement).
    const bool gx = xe || (ye && xa);
    const bool gy = ye || (xe && (topA || botA));
    if (gx) {
      if (gy) run<true, true, false>(); else run<true, false, false>();
    } else if (gy) {
      run<false, true, false>();
    } else if (a.ax == 2) {
      run<false, false, 2>();
    } else if (xa || (ADJ && (topA || botA))) {
      // x-flush windows take the own-value cross-lane moves; a window flush only in y runs the
      // edge-free body (its halo rows come from the LDS sources above), except in the
      // transposed step, whose flush rows also swap a weight
      run<false, false, true>();
    } else {
      run<false, false, false>();
    }
  }
};

// Two launch shapes.  Tile launch: one workgroup per (x, y, z-segment) tile.  Balanced launch
// (a.nwork > 0): the (column, plane) units of all x-y columns, column-major, are cut into
// nwork equal contiguous shares; a workgroup streams its share as one or more column
// segments, so every workgroup does the same work and the pipeline fill is paid once or twice
// per workgroup instead of once per short tile.
template <int K, int V, int R, int NW, bool HOT, bool ADJ, bool ACC, bool FULL, int PD>
__global__ __launch_bounds__(64 * NW) void tb3d_kernel(Tb3dArgs a) {
  using Tile = Tb3dTile<K, V, R, NW, HOT, ADJ, ACC, FULL, PD>;
  __shared__ __align__(16) float hal[2 * K * NW * 2 * 64 * V];
  __shared__ __align__(16) float qring[Tile::QR > 0 ? Tile::QR * NW * R * 64 * V : 1];
  Tile t(a, threadIdx.x & 63, __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), hal, qring);
  if (a.nwork == 0) {
    t.process(xcd_remap(blockIdx.x, a.ntx * a.nty * a.nsegz));
    return;
  }
  const int w = xcd_remap(blockIdx.x, a.nwork);
  const int nzo = a.zhi - a.zlo;  // output planes per column
  const long long units = (long long)a.ntx * a.nty * nzo;
  long long u = units * w / a.nwork;
  const long long u1 = units * (w + 1) / a.nwork;
  while (u < u1) {
    const int col = (int)(u / nzo);
    const int zs = (int)(u - (long long)col * nzo);
    const int ze = (int)min((long long)nzo, zs + (u1 - u));
    t.process_column(col % a.ntx, col / a.ntx, a.zlo + zs, a.zlo + ze);
    u += ze - zs;
  }
}
