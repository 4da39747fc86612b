/*
 * stencil_oracle.c -- plain CPU oracle for iterated first-order star stencils.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the library's product path may include, link or
 * call this file; only the test suite, the smoke check and the bench's CPU-baseline leg use
 * it.  It shares no code with the HIP library.
 *
 * What it computes (Zohouri, Podobas, Matsuoka, "Combined Spatial and Temporal Blocking for
 * High-Performance Stencil Computation on FPGAs Using OpenCL"):
 *
 *   * Section 2.1: each time step reads every cell from one buffer and writes the updated
 *     cell to a second buffer; the buffers are swapped before the next step (Jacobi
 *     ping-pong, out-of-place).
 *   * Table 2: Diffusion 2D/3D are weighted sums of the centre and the 4 (2D) or 6 (3D)
 *     face neighbours; Hotspot adds a per-cell power term scaled by sdc and an ambient
 *     temperature term.  Hotspot is evaluated in its weighted-sum form (centre and
 *     neighbour weights, plus cp*power + c_amb*t_amb); the physical Table-2 form of
 *     Hotspot 2D maps onto it with cc = 1 - sdc*(2Rx+2Ry+Rz), cw = ce = sdc*Rx,
 *     cn = cs = sdc*Ry, cp = sdc, c_amb = sdc*Rz.
 *   * Table 2, Hotspot 2D as printed (form ORACLE_HOTSPOT_PHYS, 2D only): the new value is
 *     the centre plus sdc times the sum of the power, the y-difference (n + s - 2c) times
 *     Ry_1, the x-difference (e + w - 2c) times Rx_1 and the ambient difference
 *     (TEMP_AMB - c) times Rz_1.  The coefficient vector carries sdc in cp, Rx_1 in ce,
 *     Ry_1 in cs, Rz_1 in c_amb and TEMP_AMB in t_amb; the other weights are unused.
 *   * Section 5.1: an out-of-range neighbour of a boundary cell takes the value of the
 *     boundary cell itself (clamp-to-edge), in every direction and at every step.
 *
 * Evaluation order (the paper does not fix one; this is the reading used throughout):
 *   diffusion: acc = cc*c;
 *   hotspot:   acc = fma(cc, c, q), where the time-invariant source q = fma(cp, p, k_amb)
 *              (k_amb = c_amb*t_amb rounded once in the working precision) starts the sum;
 *   then acc = fma(cw,w,acc); acc = fma(ce,e,acc); acc = fma(cs,s,acc); acc = fma(cn,n,acc);
 *   [3D: acc = fma(cb,b,acc); acc = fma(ca,a,acc)].
 *   physical Hotspot 2D, term by term in the order the formula is written:
 *              dy = (n + s) - 2c;  dx = (e + w) - 2c;  dz = TEMP_AMB - c   (each rounded);
 *              acc = fma(dy, Ry_1, p); acc = fma(dx, Rx_1, acc); acc = fma(dz, Rz_1, acc);
 *              out = fma(sdc, acc, c).
 * Two instantiations are built from the same text: FP64 (coefficients promoted from their
 * FP32 values) and FP32.  Compile with -ffp-contract=off so no other fusion happens.
 *
 * The adjoint is the literal transpose of the forward gather: every cell i scatters
 * c_d * lambda[i] onto the cell its direction-d neighbour clamps to.  With
 * x_{t+1} = A x_t + cp*p + k_amb, lambda_T = dJ/dx_T:
 *   grad_x0 = (A^T)^T lambda_T,  grad_p = cp * sum_{t=1..T} lambda_t.
 * For the physical Hotspot 2D form every occurrence of a cell in the printed formula
 * scatters its own partial derivative (1 for the leading centre, sdc*Ry_1 for n and s,
 * -2*sdc*Ry_1 for the centre inside the y-difference, and so on), and grad_p uses sdc.
 *
 * Parallelism: the forward sweep parallelises over rows with OpenMP; every output cell has
 * exactly one writer, so results do not depend on the thread count.  The adjoint scatter
 * runs serially.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

enum { ORACLE_DIFFUSION = 0, ORACLE_HOTSPOT = 1, ORACLE_HOTSPOT_PHYS = 2 };
enum { C_CC = 0, C_CW, C_CE, C_CN, C_CS, C_CB, C_CA, C_CP, C_AMB, C_TAMB };

static inline long clampl(long v, long lo, long hi) { return v < lo ? lo : (v > hi ? hi : v); }

int oracle_num_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

/* One instantiation per precision.  REAL is the working type, FMA its fused multiply-add. */
#define ORACLE_DEFINE(REAL, SUF, FMA)                                                            \
  /* Forward: T clamped Jacobi steps applied to grid (in/out).  power may be NULL for         \
   * diffusion.  Returns 0, or -1 on bad arguments / allocation failure. */                   \
  int oracle_forward_##SUF(int form, int ndim, int nx, int ny, int nz, const float* cf,       \
                           REAL* grid, const REAL* power, int T) {                            \
    if (nx < 1 || ny < 1 || nz < 1 || T < 0 || (ndim != 2 && ndim != 3)) return -1;           \
    if (ndim == 2) nz = 1;                                                                    \
    if ((form == ORACLE_HOTSPOT || form == ORACLE_HOTSPOT_PHYS) && !power) return -1;         \
    if (form == ORACLE_HOTSPOT_PHYS && ndim != 2) return -1;                                  \
    if (form < ORACLE_DIFFUSION || form > ORACLE_HOTSPOT_PHYS) return -1;                     \
    const long n = (long)nx * ny * nz;                                                        \
    const REAL cc = (REAL)cf[C_CC], cw = (REAL)cf[C_CW], ce = (REAL)cf[C_CE];                 \
    const REAL cn = (REAL)cf[C_CN], cs = (REAL)cf[C_CS], cb = (REAL)cf[C_CB];                 \
    const REAL ca = (REAL)cf[C_CA], cp = (REAL)cf[C_CP];                                      \
    const REAL kamb = (REAL)cf[C_AMB] * (REAL)cf[C_TAMB];                                     \
    /* physical Hotspot 2D: sdc, Rx_1, Ry_1, Rz_1, TEMP_AMB */                                \
    const REAL sdc = cp, rx = ce, ry = cs, rz = (REAL)cf[C_AMB], tamb = (REAL)cf[C_TAMB];     \
    REAL* buf = (REAL*)malloc(sizeof(REAL) * (size_t)n);                                      \
    REAL* q = NULL;                                                                           \
    if (!buf) return -1;                                                                      \
    if (form == ORACLE_HOTSPOT) {                                                             \
      q = (REAL*)malloc(sizeof(REAL) * (size_t)n);                                            \
      if (!q) { free(buf); return -1; }                                                       \
      for (long i = 0; i < n; ++i) q[i] = FMA(cp, power[i], kamb);                            \
    }                                                                                         \
    REAL* v = grid;                                                                           \
    REAL* o = buf;                                                                            \
    for (int t = 0; t < T; ++t) {                                                             \
      _Pragma("omp parallel for collapse(2) schedule(static)")                                \
      for (long z = 0; z < nz; ++z) {                                                         \
        for (long y = 0; y < ny; ++y) {                                                       \
          const long zm = clampl(z - 1, 0, nz - 1), zp = clampl(z + 1, 0, nz - 1);            \
          const long ym = clampl(y - 1, 0, ny - 1), yp = clampl(y + 1, 0, ny - 1);            \
          const REAL* row = v + (z * ny + y) * nx;                                            \
          const REAL* rn = v + (z * ny + ym) * nx;                                            \
          const REAL* rs = v + (z * ny + yp) * nx;                                            \
          const REAL* rb = v + (zm * ny + y) * nx;                                            \
          const REAL* ra = v + (zp * ny + y) * nx;                                            \
          REAL* out = o + (z * ny + y) * nx;                                                  \
          const REAL* qr = q ? q + (z * ny + y) * nx : NULL;                                  \
          if (form == ORACLE_HOTSPOT_PHYS) {                                                  \
            const REAL* pr = power + y * nx;                                                  \
            for (long x = 0; x < nx; ++x) {                                                   \
              const long xm = clampl(x - 1, 0, nx - 1), xp = clampl(x + 1, 0, nx - 1);        \
              const REAL c = row[x];                                                          \
              const REAL dy = (rn[x] + rs[x]) - (REAL)2 * c;                                  \
              const REAL dx = (row[xp] + row[xm]) - (REAL)2 * c;                              \
              const REAL dz = tamb - c;                                                       \
              REAL acc = FMA(dy, ry, pr[x]);                                                  \
              acc = FMA(dx, rx, acc);                                                         \
              acc = FMA(dz, rz, acc);                                                         \
              out[x] = FMA(sdc, acc, c);                                                      \
            }                                                                                 \
            continue;                                                                         \
          }                                                                                   \
          for (long x = 0; x < nx; ++x) {                                                     \
            const long xm = clampl(x - 1, 0, nx - 1), xp = clampl(x + 1, 0, nx - 1);          \
            REAL acc = qr ? FMA(cc, row[x], qr[x]) : cc * row[x];                             \
            acc = FMA(cw, row[xm], acc);                                                      \
            acc = FMA(ce, row[xp], acc);                                                      \
            acc = FMA(cs, rs[x], acc);                                                        \
            acc = FMA(cn, rn[x], acc);                                                        \
            if (ndim == 3) {                                                                  \
              acc = FMA(cb, rb[x], acc);                                                      \
              acc = FMA(ca, ra[x], acc);                                                      \
            }                                                                                 \
            out[x] = acc;                                                                     \
          }                                                                                   \
        }                                                                                     \
      }                                                                                       \
      REAL* tmp = v; v = o; o = tmp;                                                          \
    }                                                                                         \
    if (v != grid) memcpy(grid, v, sizeof(REAL) * (size_t)n);                                 \
    free(buf);                                                                                \
    free(q);                                                                                  \
    return 0;                                                                                 \
  }                                                                                           \
                                                                                              \
  /* Adjoint (vector-Jacobian product) of T forward steps.  cot = dJ/dx_T.  Writes           \
   * grad_x0 = dJ/dx_0 and, when grad_p is not NULL (hotspot), grad_p = dJ/dp.  The          \
   * affine source does not enter the adjoint, so no forward state is needed. */             \
  int oracle_adjoint_##SUF(int form, int ndim, int nx, int ny, int nz, const float* cf,       \
                           const REAL* cot, int T, REAL* grad_x0, REAL* grad_p) {             \
    if (nx < 1 || ny < 1 || nz < 1 || T < 0 || (ndim != 2 && ndim != 3)) return -1;           \
    if (ndim == 2) nz = 1;                                                                    \
    if (form < ORACLE_DIFFUSION || form > ORACLE_HOTSPOT_PHYS) return -1;                     \
    if (form == ORACLE_HOTSPOT_PHYS && ndim != 2) return -1;                                  \
    const long n = (long)nx * ny * nz;                                                        \
    const REAL cc = (REAL)cf[C_CC], cw = (REAL)cf[C_CW], ce = (REAL)cf[C_CE];                 \
    const REAL cn = (REAL)cf[C_CN], cs = (REAL)cf[C_CS], cb = (REAL)cf[C_CB];                 \
    const REAL ca = (REAL)cf[C_CA], cp = (REAL)cf[C_CP];                                      \
    const REAL sdc = cp, rx = ce, ry = cs, rz = (REAL)cf[C_AMB];                              \
    REAL* lam = grad_x0;                                                                      \
    REAL* nl = (REAL*)malloc(sizeof(REAL) * (size_t)n);                                       \
    if (!nl) return -1;                                                                       \
    memcpy(lam, cot, sizeof(REAL) * (size_t)n);                                               \
    if (grad_p) memset(grad_p, 0, sizeof(REAL) * (size_t)n);                                  \
    for (int t = T; t >= 1; --t) {                                                            \
      if (grad_p && form != ORACLE_DIFFUSION)                                                 \
        for (long i = 0; i < n; ++i) grad_p[i] = grad_p[i] + cp * lam[i];                     \
      memset(nl, 0, sizeof(REAL) * (size_t)n);                                                \
      for (long z = 0; z < nz; ++z)                                                           \
        for (long y = 0; y < ny; ++y)                                                         \
          for (long x = 0; x < nx; ++x) {                                                     \
            const REAL l = lam[(z * ny + y) * nx + x];                                        \
            if (form == ORACLE_HOTSPOT_PHYS) {                                                \
              const long i = y * nx + x;                                                      \
              const REAL g = sdc * l;                                                         \
              nl[i] += l;                                                                     \
              nl[clampl(y - 1, 0, ny - 1) * nx + x] += ry * g;                                \
              nl[clampl(y + 1, 0, ny - 1) * nx + x] += ry * g;                                \
              nl[i] += -2 * ry * g;                                                           \
              nl[y * nx + clampl(x + 1, 0, nx - 1)] += rx * g;                                \
              nl[y * nx + clampl(x - 1, 0, nx - 1)] += rx * g;                                \
              nl[i] += -2 * rx * g;                                                           \
              nl[i] += -rz * g;                                                               \
              continue;                                                                       \
            }                                                                                 \
            nl[(z * ny + y) * nx + x] += cc * l;                                              \
            nl[(z * ny + y) * nx + clampl(x - 1, 0, nx - 1)] += cw * l;                       \
            nl[(z * ny + y) * nx + clampl(x + 1, 0, nx - 1)] += ce * l;                       \
            nl[(z * ny + clampl(y + 1, 0, ny - 1)) * nx + x] += cs * l;                       \
            nl[(z * ny + clampl(y - 1, 0, ny - 1)) * nx + x] += cn * l;                       \
            if (ndim == 3) {                                                                  \
              nl[(clampl(z - 1, 0, nz - 1) * ny + y) * nx + x] += cb * l;                     \
              nl[(clampl(z + 1, 0, nz - 1) * ny + y) * nx + x] += ca * l;                     \
            }                                                                                 \
          }                                                                                   \
      memcpy(lam, nl, sizeof(REAL) * (size_t)n);                                              \
    }                                                                                         \
    free(nl);                                                                                 \
    return 0;                                                                                 \
  }

ORACLE_DEFINE(double, f64, fma)
ORACLE_DEFINE(float, f32, fmaf)

/*
 * Radius-r star stencil in 2D, diffusion form (Eq. 1 and Eq. 2 are written for a general
 * radius rad; Table 2's stencils are its rad = 1 case).  Each cell is updated from itself and
 * the cells at distance d = 1..rad along each axis:
 *   out = cc*c + sum_d (w_d*[x-d] + e_d*[x+d]) + sum_d s_d*[y+d] + sum_d n_d*[y-d]
 * The clamp of Section 5.1 extends to every distance: an index beyond the grid is replaced
 * by the nearest boundary index (the neighbour takes the boundary cell's value).
 * Weight layout (1 + 4*rad floats), which is also the evaluation order of the FMA chain:
 *   wts[0] = cc; for d = 1..rad: wts[2d-1] = w_d, wts[2d] = e_d;
 *   wts[2rad+d] = s_d (d = 1..rad); wts[3rad+d] = n_d (d = 1..rad).
 * With rad = 1 this is the chain c, w, e, s, n of the radius-1 diffusion forward above.
 * Hotspot form (oracle_star2d_src_*, power non-NULL): the radius-1 hotspot source carried over
 * to radius r, q = fma(cp, p, c_amb*t_amb) per cell (src = {cp, c_amb, t_amb}, c_amb*t_amb
 * rounded once in the working precision) and the chain starts from fma(cc, c, q), as the
 * radius-1 hotspot forward does; power NULL is the diffusion form.
 */
#define ORACLE_STAR_DEFINE(REAL, SUF, FMA)                                                       \
  int oracle_star2d_src_##SUF(int rad, int nx, int ny, const float* wts, const float* src,      \
                              const REAL* power, REAL* grid, int T) {                          \
    if (rad < 1 || nx < 1 || ny < 1 || T < 0) return -1;                                       \
    const long n = (long)nx * ny;                                                              \
    REAL* buf = (REAL*)malloc(sizeof(REAL) * (size_t)n);                                       \
    REAL* q = power ? (REAL*)malloc(sizeof(REAL) * (size_t)n) : NULL;                          \
    if (!buf || (power && !q)) { free(buf); free(q); return -1; }                              \
    if (power) {                                                                               \
      const REAL kamb = (REAL)src[1] * (REAL)src[2];                                           \
      for (long i = 0; i < n; ++i) q[i] = FMA((REAL)src[0], power[i], kamb);                   \
    }                                                                                          \
    REAL* v = grid;                                                                            \
    REAL* o = buf;                                                                             \
    for (int t = 0; t < T; ++t) {                                                              \
      _Pragma("omp parallel for schedule(static)")                                             \
      for (long y = 0; y < ny; ++y) {                                                          \
        const REAL* row = v + y * nx;                                                          \
        for (long x = 0; x < nx; ++x) {                                                        \
          REAL acc = q ? FMA((REAL)wts[0], row[x], q[y * nx + x]) : (REAL)wts[0] * row[x];     \
          for (int d = 1; d <= rad; ++d) {                                                     \
            acc = FMA((REAL)wts[2 * d - 1], row[clampl(x - d, 0, nx - 1)], acc);               \
            acc = FMA((REAL)wts[2 * d], row[clampl(x + d, 0, nx - 1)], acc);                   \
          }                                                                                    \
          for (int d = 1; d <= rad; ++d)                                                       \
            acc = FMA((REAL)wts[2 * rad + d], v[clampl(y + d, 0, ny - 1) * nx + x], acc);      \
          for (int d = 1; d <= rad; ++d)                                                       \
            acc = FMA((REAL)wts[3 * rad + d], v[clampl(y - d, 0, ny - 1) * nx + x], acc);      \
          o[y * nx + x] = acc;                                                                 \
        }                                                                                      \
      }                                                                                        \
      REAL* tmp = v; v = o; o = tmp;                                                           \
    }                                                                                          \
    if (v != grid) memcpy(grid, v, sizeof(REAL) * (size_t)n);                                  \
    free(buf);                                                                                 \
    free(q);                                                                                   \
    return 0;                                                                                  \
  }                                                                                            \
  int oracle_star2d_##SUF(int rad, int nx, int ny, const float* wts, REAL* grid, int T) {       \
    return oracle_star2d_src_##SUF(rad, nx, ny, wts, NULL, NULL, grid, T);                     \
  }

ORACLE_STAR_DEFINE(double, f64, fma)
ORACLE_STAR_DEFINE(float, f32, fmaf)

/*
 * Radius-r star stencil in 3D, diffusion form (Eq. 1 and Eq. 2 are written for a general rad
 * in both 2D and 3D; the 3D shift register of Eq. 1 spans 2*rad planes).  Each cell is updated
 * from itself and the cells at distance d = 1..rad along each of the three axes:
 *   out = cc*c + sum_d (w_d*[x-d] + e_d*[x+d]) + sum_d s_d*[y+d] + sum_d n_d*[y-d]
 *               + sum_d b_d*[z-d] + sum_d a_d*[z+d]
 * with the clamp of Section 5.1 at every distance (an index beyond the grid is replaced by the
 * nearest boundary index).
 * Weight layout (1 + 6*rad floats), which is also the evaluation order of the FMA chain:
 *   wts[0] = cc; for d = 1..rad: wts[2d-1] = w_d, wts[2d] = e_d;
 *   wts[2rad+d] = s_d; wts[3rad+d] = n_d; wts[4rad+d] = b_d; wts[5rad+d] = a_d (d = 1..rad).
 * With rad = 1 this is the chain c, w, e, s, n, b, a of the radius-1 3D forward above.
 * Hotspot form (oracle_star3d_src_*): as for 2D, the chain starts from fma(cc, c, q).
 */
#define ORACLE_STAR3_DEFINE(REAL, SUF, FMA)                                                      \
  int oracle_star3d_src_##SUF(int rad, int nx, int ny, int nz, const float* wts, const float* src, \
                              const REAL* power, REAL* grid, int T) {                          \
    if (rad < 1 || nx < 1 || ny < 1 || nz < 1 || T < 0) return -1;                             \
    const long n = (long)nx * ny * nz;                                                         \
    REAL* buf = (REAL*)malloc(sizeof(REAL) * (size_t)n);                                       \
    REAL* q = power ? (REAL*)malloc(sizeof(REAL) * (size_t)n) : NULL;                          \
    if (!buf || (power && !q)) { free(buf); free(q); return -1; }                              \
    if (power) {                                                                               \
      const REAL kamb = (REAL)src[1] * (REAL)src[2];                                           \
      for (long i = 0; i < n; ++i) q[i] = FMA((REAL)src[0], power[i], kamb);                   \
    }                                                                                          \
    REAL* v = grid;                                                                            \
    REAL* o = buf;                                                                             \
    for (int t = 0; t < T; ++t) {                                                              \
      _Pragma("omp parallel for collapse(2) schedule(static)")                                 \
      for (long z = 0; z < nz; ++z) {                                                          \
        for (long y = 0; y < ny; ++y) {                                                        \
          const REAL* row = v + (z * ny + y) * nx;                                             \
          for (long x = 0; x < nx; ++x) {                                                      \
            const long ic = (z * ny + y) * nx + x;                                             \
            REAL acc = q ? FMA((REAL)wts[0], row[x], q[ic]) : (REAL)wts[0] * row[x];           \
            for (int d = 1; d <= rad; ++d) {                                                   \
              acc = FMA((REAL)wts[2 * d - 1], row[clampl(x - d, 0, nx - 1)], acc);             \
              acc = FMA((REAL)wts[2 * d], row[clampl(x + d, 0, nx - 1)], acc);                 \
            }                                                                                  \
            for (int d = 1; d <= rad; ++d)                                                     \
              acc = FMA((REAL)wts[2 * rad + d], v[(z * ny + clampl(y + d, 0, ny - 1)) * nx + x], acc); \
            for (int d = 1; d <= rad; ++d)                                                     \
              acc = FMA((REAL)wts[3 * rad + d], v[(z * ny + clampl(y - d, 0, ny - 1)) * nx + x], acc); \
            for (int d = 1; d <= rad; ++d)                                                     \
              acc = FMA((REAL)wts[4 * rad + d], v[(clampl(z - d, 0, nz - 1) * ny + y) * nx + x], acc); \
            for (int d = 1; d <= rad; ++d)                                                     \
              acc = FMA((REAL)wts[5 * rad + d], v[(clampl(z + d, 0, nz - 1) * ny + y) * nx + x], acc); \
            o[ic] = acc;                                                                       \
          }                                                                                    \
        }                                                                                      \
      }                                                                                        \
      REAL* tmp = v; v = o; o = tmp;                                                           \
    }                                                                                          \
    if (v != grid) memcpy(grid, v, sizeof(REAL) * (size_t)n);                                  \
    free(buf);                                                                                 \
    free(q);                                                                                   \
    return 0;                                                                                  \
  }                                                                                            \
  int oracle_star3d_##SUF(int rad, int nx, int ny, int nz, const float* wts, REAL* grid, int T) { \
    return oracle_star3d_src_##SUF(rad, nx, ny, nz, wts, NULL, NULL, grid, T);                 \
  }

ORACLE_STAR3_DEFINE(double, f64, fma)
ORACLE_STAR3_DEFINE(float, f32, fmaf)

/*
 * Adjoint of T steps of the radius-r star stencil (2D: nz = 1; both forms share it, the source
 * being independent of the state): lam holds lambda_T = dJ/dx_T on entry and dJ/dx_0 on exit.
 * Each step scatters every term of the forward update: the cell's own weight cc, and each
 * directional weight to the neighbour index the forward step read, clamped as in Section 5.1
 * (so the weights of out-of-grid neighbours land on the boundary cell):
 *   lambda_{t-1}[clamp(i + offset)] += weight * lambda_t[i]   for every term of cell i.
 * With grad_p non-NULL (the hotspot form): grad_p = cp * sum_{t=1..T} lambda_t.
 * Weights in the layout of oracle_star2d (2D) or oracle_star3d (3D).
 */
#define ORACLE_STAR_ADJ_DEFINE(REAL, SUF)                                                        \
  int oracle_star_adjoint_##SUF(int ndim, int rad, int nx, int ny, int nz, const float* wts,     \
                                float cp, REAL* lam, int T, REAL* grad_p) {                    \
    if ((ndim != 2 && ndim != 3) || rad < 1 || nx < 1 || ny < 1 || nz < 1 || T < 0) return -1;  \
    if (ndim == 2) nz = 1;                                                                     \
    const long n = (long)nx * ny * nz;                                                         \
    REAL* nxt = (REAL*)malloc(sizeof(REAL) * (size_t)n);                                       \
    if (!nxt) return -1;                                                                       \
    if (grad_p)                                                                                \
      for (long i = 0; i < n; ++i) grad_p[i] = 0;                                              \
    for (int t = T; t >= 1; --t) {                                                             \
      if (grad_p)                                                                              \
        for (long i = 0; i < n; ++i) grad_p[i] = grad_p[i] + (REAL)cp * lam[i];                \
      for (long i = 0; i < n; ++i) nxt[i] = 0;                                                 \
      for (long z = 0; z < nz; ++z)                                                            \
        for (long y = 0; y < ny; ++y)                                                          \
          for (long x = 0; x < nx; ++x) {                                                      \
            const long i = (z * ny + y) * nx + x;                                              \
            const REAL l = lam[i];                                                             \
            nxt[i] += (REAL)wts[0] * l;                                                        \
            for (int d = 1; d <= rad; ++d) {                                                   \
              nxt[(z * ny + y) * nx + clampl(x - d, 0, nx - 1)] += (REAL)wts[2 * d - 1] * l;   \
              nxt[(z * ny + y) * nx + clampl(x + d, 0, nx - 1)] += (REAL)wts[2 * d] * l;       \
              nxt[(z * ny + clampl(y + d, 0, ny - 1)) * nx + x] += (REAL)wts[2 * rad + d] * l; \
              nxt[(z * ny + clampl(y - d, 0, ny - 1)) * nx + x] += (REAL)wts[3 * rad + d] * l; \
              if (ndim == 3) {                                                                 \
                nxt[(clampl(z - d, 0, nz - 1) * ny + y) * nx + x] += (REAL)wts[4 * rad + d] * l; \
                nxt[(clampl(z + d, 0, nz - 1) * ny + y) * nx + x] += (REAL)wts[5 * rad + d] * l; \
              }                                                                                \
            }                                                                                  \
          }                                                                                    \
      memcpy(lam, nxt, sizeof(REAL) * (size_t)n);                                              \
    }                                                                                          \
    free(nxt);                                                                                 \
    return 0;                                                                                  \
  }

ORACLE_STAR_ADJ_DEFINE(double, f64)
ORACLE_STAR_ADJ_DEFINE(float, f32)
