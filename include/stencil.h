/*
 * stencil.h -- C ABI of the MI355X (gfx950) temporal-blocked star-stencil library.
 *
 * The library runs T time steps of first-order star stencils (5-point 2D, 7-point 3D) in
 * FP32 on one GPU, with combined spatial and temporal blocking: overlapped tiles carry
 * several fused time steps per pass over HBM.  Method: Zohouri, Podobas, Matsuoka,
 * "Combined Spatial and Temporal Blocking for High-Performance Stencil Computation on FPGAs
 * Using OpenCL" (Sections 2.1, 3.1, 3.2, 4, 5.1; Table 2).
 *
 * Conventions shared by every entry point
 *   - Grids are FP32, row-major, x fastest: index = (z*ny + y)*nx + x (2D: nz = 1).
 *   - Directions: w = x-1, e = x+1, n = y-1, s = y+1, b = z-1, a = z+1.
 *   - Boundary: an out-of-range neighbour takes the value of the boundary cell itself, in
 *     every direction and at every step (Section 5.1).
 *   - One time step (Section 2.1, Table 2) reads every cell from one buffer and writes
 *       out = cc*c + cw*w + ce*e + cs*s + cn*n [+ cb*b + ca*a]   (diffusion)
 *       out = q + (same weighted sum),  q = fma(cp, p, c_amb*t_amb)  (hotspot)
 *     evaluated as the FMA chain c, w, e, s, n, b, a; for hotspot the chain starts from
 *     fma(cc, c, q), with k_amb = c_amb*t_amb rounded once in FP32.  Steps are Jacobi
 *     (out-of-place, ping-pong).
 *   - Pointers named "device" must be device memory of the current HIP device, 16-byte
 *     aligned for the fast path (4-byte aligned is accepted), and must not alias each
 *     other.  The caller owns them and keeps them alive until the stream work completes.
 *   - Every call is stream-ordered on the plan's stream (or the stream passed in); nothing
 *     synchronises the host unless stated.
 *   - Errors: argument errors return before any device work.  No C++ exception crosses
 *     this ABI.  stencil_last_error() gives a thread-local detail message.
 */
#ifndef STENCIL_MI355_H
#define STENCIL_MI355_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  STENCIL_OK = 0,
  STENCIL_ERR_INVALID_ARG = -1,   /* bad pointer, size, step count, coefficient, form */
  STENCIL_ERR_UNSUPPORTED = -2,   /* valid request the library does not implement */
  STENCIL_ERR_OUT_OF_MEMORY = -3, /* device allocation of plan-owned memory failed */
  STENCIL_ERR_HIP = -4,           /* a HIP runtime call failed (message in stencil_last_error) */
  STENCIL_ERR_INTERNAL = -5       /* invariant violated inside the library */
} stencil_status_t;

/* HOTSPOT is the weighted-sum form above.  HOTSPOT_PHYS (2D only) is Table 2's Hotspot 2D
 * formula as printed,
 *     out = c + sdc*(p + ((n + s) - 2c)*Ry_1 + ((e + w) - 2c)*Rx_1 + (TEMP_AMB - c)*Rz_1),
 * every operation rounded in FP32 in that order, each "x + y*z" as one FMA and the final
 * c + sdc*(...) as fma(sdc, ..., c).  A field at TEMP_AMB with zero power is then an exact
 * fixed point.  Its linear part is symmetric, so stencil_adjoint applies the same formula
 * with no power and TEMP_AMB = 0 as the transposed step.  It has no batched launch
 * (UNSUPPORTED). */
typedef enum { STENCIL_DIFFUSION = 0, STENCIL_HOTSPOT = 1, STENCIL_HOTSPOT_PHYS = 2 } stencil_form_t;

/* Stencil weights (Table 2).  cb, ca are ignored for 2D; cp, c_amb, t_amb for diffusion.
 * All must be finite.  The paper's Hotspot 2D form maps onto these with
 * cc = 1 - sdc*(2Rx_1 + 2Ry_1 + Rz_1), cw = ce = sdc*Rx_1, cn = cs = sdc*Ry_1, cp = sdc,
 * c_amb = sdc*Rz_1; its Hotspot 3D form sets c_amb = ca.
 * HOTSPOT_PHYS reads its parameters from the same struct: sdc from cp, Rx_1 from ce, Ry_1
 * from cs, Rz_1 from c_amb and TEMP_AMB from t_amb; the other fields are ignored. */
typedef struct {
  float cc, cw, ce, cn, cs, cb, ca;
  float cp;    /* hotspot: weight of the power map (sdc in Table 2) */
  float c_amb; /* hotspot: ambient coupling */
  float t_amb; /* hotspot: ambient temperature (a compile-time constant in the paper) */
} stencil_coeffs_t;

/* Blocking parameters.  0 in any field means "choose automatically".
 *   variant  0 auto, 1 plain one-step-per-pass kernel, 2 temporal-blocked kernel
 *   k        fused time steps per pass (par_time of Section 3.2; halo = k, Eq. 2)
 *   vec      FP32 cells per lane along x (par_vec of Section 3.1)
 *   bsize_x  spatial block width in cells (64*vec for the temporal-blocked kernels)
 *   bsize_y  3D: spatial block height in cells
 *   seg_len  cells of the streamed axis (y in 2D, z in 3D) handled by one tile pass
 *   nwork    3D: workgroups of the balanced launch, where each workgroup streams an equal share
 *            of all x-y columns' planes (reported: 0 means the tile launch, one workgroup per
 *            tile of seg_len planes).  As input, nwork > 0 selects the balanced launch with that
 *            many workgroups; 0 leaves the choice to the tuner (or, with seg_len > 0, to the tile
 *            launch). */
typedef struct {
  int variant, k, vec, bsize_x, bsize_y, seg_len, nwork;
} stencil_tuning_t;

typedef struct stencil_plan_s* stencil_plan_t;

/* Create a plan for a grid of nx*ny*nz cells (ndim 2: nz must be 1).  The plan fixes the
 * blocking of Sections 3.1-3.2: spatial blocks overlapping by a halo of k cells per side
 * (Eq. 2, 4, 5) that stream along the outermost axis and carry k fused time steps per pass.
 * Allocates the plan's ping-pong scratch (one grid) on the current device and, when tuning is
 * NULL or has zero fields, picks k and the block shape as Section 5.3 does: the
 * bandwidth/halo cost model (Section 4) prunes the candidates and short timed trials on
 * scratch memory decide among the best (cached per shape).  hip_stream: a hipStream_t, or
 * NULL for the default stream.  *out receives the plan; on error *out is NULL. */
stencil_status_t stencil_create(stencil_plan_t* out, stencil_form_t form, int ndim, int nx, int ny,
                                int nz, const stencil_tuning_t* tuning, void* hip_stream);

/* Run exactly T >= 0 time steps in place on grid (device, nx*ny*nz FP32).  power (device,
 * same shape) is required for both hotspot forms and ignored for DIFFUSION.  T == 0 leaves grid
 * unchanged.  Enqueues ceil(T/k) temporal-blocked passes (the last one shorter when k does
 * not divide T, Section 3.2) alternating between grid and plan scratch so that the result
 * lands in grid.  Asynchronous. */
stencil_status_t stencil_run(stencil_plan_t plan, float* grid, const float* power,
                             const stencil_coeffs_t* coeffs, int T);

/* As stencil_run, and additionally keeps checkpoints of the field every ckpt_every steps
 * (0 = round(sqrt(T))) in plan-owned device memory: checkpoint j holds x_{j*ckpt_every}
 * for j = 0 .. floor((T-1)/ckpt_every).  Passes are cut at checkpoint steps.  The
 * checkpoints replace any earlier ones.  Returns OUT_OF_MEMORY if they do not fit. */
stencil_status_t stencil_run_ckpt(stencil_plan_t plan, float* grid, const float* power,
                                  const stencil_coeffs_t* coeffs, int T, int ckpt_every);

/* One temporal-blocked pass over a slab whose faces along the streamed axis (z in 3D, y in 2D)
 * may be ghost faces: the spatial blocking of Sections 3.1-3.2 lifted to a whole device, where
 * a grid too large for one device is cut into slabs along the streamed axis and each slab
 * carries copies of its neighbours' cells (Section 1 motivates spatial blocking by exactly
 * this distribution of large inputs; Section 8 names multi-device distribution as future work).
 * The plan's grid is the slab with its ghost planes: the first ghost_lo and the last ghost_hi
 * planes (rows in 2D) are ghost planes, supplied by the caller; a depth of 0 marks a true grid
 * face, which is clamped (Section 5.1).  Runs T fused steps from src to dst (both device,
 * plan-shaped, out of place) in one pass and writes only the interior planes
 * [ghost_lo, n - ghost_hi) of dst; dst's ghost planes are not written.  The interior then
 * equals T steps of the whole grid restricted to the slab, because a step moves information
 * one plane, so the far side of a ghost region (where the slab array ends) reaches at most T
 * planes inward.  Requires T <= every non-zero ghost depth (INVALID_ARG) and T <= the largest
 * fused step count of the kernels (UNSUPPORTED beyond it: 24 for 2D diffusion, 16 for 2D
 * hotspot, 6 for 3D diffusion, 4 for 3D hotspot); T = 0 copies the interior.  power (hotspot)
 * is the slab's power map with the same ghost planes.  Not for plain (variant 1) or star
 * plans (UNSUPPORTED).  Asynchronous on the plan's stream.  A multi-device run alternates
 * this pass with an exchange of the ghost planes between neighbouring slabs. */
stencil_status_t stencil_run_slab(stencil_plan_t plan, const float* src, float* dst, const float* power,
                                  const stencil_coeffs_t* coeffs, int T, int ghost_lo, int ghost_hi);

/* Adjoint (vector-Jacobian product) of T steps.  cotangent = dJ/dx_T (device, read only).
 * Writes grad_x0 = dJ/dx_0 (device) and, if grad_power is not NULL and the plan is
 * HOTSPOT, grad_power = dJ/dp (device).  Applies the transposed stencil backward in time
 * with the same temporal blocking as the forward pass; dJ/dp = cp * sum_{t=1..T} lambda_t is
 * accumulated in registers over the fused steps of a pass and written once per pass.
 * recompute = 1 additionally re-runs each checkpoint segment of the last stencil_run_ckpt
 * (power must then be the same device map) and checks the recomputed segment end equals
 * the next stored checkpoint bit for bit (STENCIL_ERR_INTERNAL if not); the gradient of
 * these affine maps does not depend on forward states, so recompute = 0 is exact too.
 * grad_x0 and grad_power must not alias cotangent. */
stencil_status_t stencil_adjoint(stencil_plan_t plan, const float* cotangent, const float* power,
                                 const stencil_coeffs_t* coeffs, int T, float* grad_x0,
                                 float* grad_power, int recompute);

/* One grid of a batch. */
typedef struct {
  stencil_form_t form; /* DIFFUSION only (the hotspot forms return UNSUPPORTED) */
  int ndim, nx, ny, nz;
  float* grid;         /* device, in/out */
  const float* power;  /* unused for diffusion */
  stencil_coeffs_t coeffs;
  int T;
} stencil_batch_item_t;

/* Opaque captured batch (persistent kernels inside a HIP graph, plus their work lists). */
typedef struct stencil_batch_s* stencil_batch_t;

/* Run every item of the batch, each for its own T steps, in one persistent launch per
 * dimensionality, captured once in a HIP graph.  Work items (grid, pass, tile) are claimed
 * in a global dependency order by resident workgroups; an item waits only for the tiles of
 * the previous pass of its own grid that overlap its halo.  The persistent kernels fuse up to
 * 16 (2D) or 4 (3D) steps per pass (256-column windows; 128 x 48 windows); each grid's T steps
 * are spread evenly over the fewest even number of passes, since a pass costs the same for any
 * number of fused steps up to the kernel's capacity.  Segment lengths (rows, planes) are chosen
 * per grid from a work model so that no grid's chain of dependent passes outlasts the
 * balanced share of the batch, and work items are claimed longest-chain first.
 *   graph_cache: NULL -> build, run and free everything in this call.
 *                non-NULL -> if *graph_cache is NULL, build and store the captured batch
 *                there; otherwise replay *graph_cache, which must have been built from
 *                items with identical shapes, T, grid pointers and coefficients
 *                (INVALID_ARG otherwise).
 * Every dependency wait is bounded: a wait that exceeds its bound (a scheduling fault) ends
 * with STENCIL_ERR_INTERNAL instead of a hang (see stencil_batch_sync for replays).
 * Items must not share grid memory.  Asynchronous on hip_stream when graph_cache is not NULL;
 * the uncached call synchronises and returns the launch's status. */
stencil_status_t stencil_run_batched(int n, const stencil_batch_item_t* items, void* hip_stream,
                                     stencil_batch_t* graph_cache);

/* Wait for the latest replay of a captured batch and report it: STENCIL_ERR_INTERNAL when a
 * dependency wait of any replay so far exceeded its bound (a scheduling fault: the results are
 * invalid and the batch should be destroyed), else OK.  A replay also reports, without
 * waiting, such a failure of an earlier replay that has completed; the uncached call reports
 * its own. */
stencil_status_t stencil_batch_sync(stencil_batch_t batch);

/* Free a captured batch (synchronises its stream first).  NULL is a no-op. */
void stencil_batch_destroy(stencil_batch_t batch);

/* The uncached stencil_run_batched for callers that cannot allocate device memory (code that
 * must not call hipMalloc, such as tight serving loops).  It allocates nothing: the caller
 * passes, besides the items, partners[i], a device buffer of item i's size that serves as
 * its ping-pong partner (contents unspecified on return; it must not alias any grid or other
 * partner); the grid table, work lists, pass flags and counters live in a fixed device array
 * of 8 MiB that each GPU holds until the process ends.  Batches whose tables exceed it return
 * INVALID_ARG.  Same results as stencil_run_batched, bit for bit.  Synchronous: it returns
 * after the batch has run on hip_stream, with STENCIL_ERR_INTERNAL if a dependency wait
 * exceeded its bound.  Calls on one GPU share the array: calls of this process are serialised
 * by a lock, calls that overlap from other processes race.  No graph is captured. */
stencil_status_t stencil_run_batched_noalloc(int n, const stencil_batch_item_t* items, float* const* partners,
                                             void* hip_stream);

/* Report the blocking the plan resolved to (after auto-tuning). */
stencil_status_t stencil_get_tuning(stencil_plan_t plan, stencil_tuning_t* out);

/* The blocking of the plan's transposed (adjoint) passes, which the tuner chooses and times on
 * their own (they also read and write grad_p): k, seg_len, nwork and the window as in
 * stencil_get_tuning.  UNSUPPORTED for star plans. */
stencil_status_t stencil_get_adjoint_tuning(stencil_plan_t plan, stencil_tuning_t* out);

/* The library's own time model for T steps of the plan's resolved blocking, the model the
 * tuner ranks candidates with: the paper's external-memory count (Section 4, Eq. 6-8, with
 * the GPU tile's halo rows added and the HBM rate at an achievable fraction of its peak)
 * next to an arithmetic term for the redundantly computed halo cells, priced per pass as the
 * larger of the two plus a launch overhead.  Host arithmetic only; no device work.
 *   seconds       modelled time of the T steps
 *   mem_seconds   memory part, summed over the passes
 *   alu_seconds   arithmetic part, summed over the passes (0 for the plain kernel)
 *   passes        passes over HBM (T for the plain one-step kernel)
 * Returns INVALID_ARG for a NULL argument or T < 0. */
typedef struct {
  double seconds, mem_seconds, alu_seconds;
  long passes;
} stencil_plan_model_t;
stencil_status_t stencil_plan_model(stencil_plan_t plan, int T, stencil_plan_model_t* out);

/* Free the plan, its scratch and checkpoints (synchronises the plan stream).  NULL ok. */
void stencil_destroy(stencil_plan_t plan);

const char* stencil_status_string(stencil_status_t status);
const char* stencil_last_error(void); /* thread-local; "" if none */

/* ---------------------------------------------------------------- radius-r star stencils
 * Eq. 1 and Eq. 2 are written for a general radius rad in 2D and 3D; Table 2's stencils are
 * rad = 1.  A radius-r star stencil (diffusion form) updates each cell from itself and the
 * cells at distance d = 1..r along each axis:
 *     out = cc*c + sum_d (w_d*[x-d] + e_d*[x+d]) + sum_d s_d*[y+d] + sum_d n_d*[y-d]
 *                [ + sum_d b_d*[z-d] + sum_d a_d*[z+d] ]                       (3D)
 * An index beyond the grid is replaced by the nearest boundary index at every distance and
 * every step (Section 5.1).  Tiles overlap by a halo of r*k cells per side: 2D tiles are
 * 256-column windows streamed along y, 3D tiles 64 x 64 x-y windows streamed along z.
 *
 * stencil_create_star: a plan for an nx*ny grid (ndim 2, nz 1) or an nx*ny*nz grid (ndim 3),
 * 1 <= rad <= 4 (larger rad returns UNSUPPORTED).  tuning as for stencil_create (seg_len is
 * the rows per tile in 2D, the planes per tile in 3D); with k == 0 the fused step count is
 * chosen by timing each instantiated k on plan scratch.  Instantiated k: 2D rad 1: 1, 2, 4, 8;
 * rad 2: 1, 2, 4, 5, 8; rad 3, 4: 1, 2, 4.  3D rad 1: 1, 2, 3; rad 2, 3: 1, 2; rad 4: 1.  A
 * larger k is lowered to the largest instantiated one.  The plan serves stencil_run_star,
 * stencil_get_tuning, stencil_plan_model (its passes priced with a halo of rad*k) and
 * stencil_destroy; stencil_run, stencil_run_ckpt and stencil_adjoint reject it.
 *
 * stencil_run_star: exactly T >= 0 steps in place on grid (device, FP32, the plan's shape).
 * weights is a HOST array of finite floats in the stencil's FMA evaluation order: cc; then
 * w_d, e_d for d = 1..rad; then s_1..s_rad; then n_1..n_rad; in 3D then b_1..b_rad and
 * a_1..a_rad.  That is 1 + 4*rad floats in 2D and 1 + 6*rad in 3D (rad = 1 gives the chain c,
 * w, e, s, n[, b, a] of stencil_run).  Asynchronous on the plan's stream. */
stencil_status_t stencil_create_star(stencil_plan_t* out, int ndim, int rad, int nx, int ny, int nz,
                                     const stencil_tuning_t* tuning, void* hip_stream);
stencil_status_t stencil_run_star(stencil_plan_t plan, float* grid, const float* weights, int T);

/* stencil_run_star_hotspot: the hotspot form of the radius-r star stencil on a star plan (2D or
 * 3D): Table 2's Hotspot source carried over to radius r, i.e. every step is
 *     out = q + (the weighted sum of stencil_run_star),  q = cp*p + c_amb*t_amb,
 * evaluated as the chain fma(cc, c, q), then the neighbour terms in stencil_run_star's order,
 * with q = fma(cp, p, k_amb) and k_amb = c_amb*t_amb rounded once in FP32 (as stencil_run's
 * hotspot form).  power: device, the grid's shape, FP32, 4-byte aligned, not aliasing grid;
 * read only.  src: HOST array {cp, c_amb, t_amb}, finite.  weights, T, grid and the stream as
 * for stencil_run_star; the plan's tuning (k, seg_len) serves both forms.  INVALID_ARG for a
 * NULL power or src, non-finite values or a non-star plan. */
stencil_status_t stencil_run_star_hotspot(stencil_plan_t plan, float* grid, const float* power, const float* weights,
                                          const float* src, int T);

/* stencil_adjoint_star: adjoint (vector-Jacobian product) of T steps of a star plan's stencil,
 * 2D or 3D, either form (the source term does not depend on the state).  cotangent = dJ/dx_T
 * (device, read only); writes grad_x0 = dJ/dx_0 (device) and, if grad_power is not NULL (the
 * hotspot form; src = {cp, c_amb, t_amb} is then required), grad_power = dJ/dp =
 * cp * sum_{t=1..T} lambda_t (device, overwritten).  Each step applies the transposed stencil
 * lambda_{t-1} = A^T lambda_t, where A is the forward step with the clamp of Section 5.1 at every
 * distance: cell j gathers the mirrored weights of the cells whose clamped neighbour it is,
 * zero beyond the grid, and a boundary cell the sum over every cell within the distance whose
 * neighbour clamps onto it.  One launch per step (not temporal-blocked).  weights as for
 * stencil_run_star.  Buffers 4-byte aligned; grad_x0 and grad_power must not alias cotangent or
 * each other.  Asynchronous on the plan's stream; uses the plan's scratch. */
stencil_status_t stencil_adjoint_star(stencil_plan_t plan, const float* cotangent, const float* weights,
                                      const float* src, int T, float* grad_x0, float* grad_power);

/* ---------------------------------------------------------------- performance model
 * The paper's external-memory model (Section 4, Eq. 3-9), as used to prune the tuning
 * space (Section 5.3).  Pure host arithmetic; needs no device.  rad = 1 for the evaluated
 * stencils.  dims: 2D uses dim_x, dim_y; 3D uses dim_x, dim_y, dim_z.  th_max in GB/s
 * (1 GB = 1e9 B). */
typedef struct {
  int ndim, rad, par_vec, par_time;
  double f_max_hz;
  int size_cell, num_read, num_write;
  int bsize_x, bsize_y;
  long dim_x, dim_y, dim_z;
  long iter;
  double th_max_gbs;
} stencil_model_params_t;

typedef struct {
  double th_mem_gbs;     /* Eq. 3 */
  long csize_x, csize_y; /* Eq. 4 */
  long bnum_x, bnum_y;   /* Eq. 5 */
  double t_cell;         /* Eq. 6 */
  double t_read, t_write;/* Eq. 7 and the write count */
  double run_time_s;     /* Eq. 8 */
  double throughput_gbs; /* Eq. 9, effective GB/s */
} stencil_model_result_t;

stencil_status_t stencil_model_estimate(const stencil_model_params_t* p, stencil_model_result_t* r);

#ifdef __cplusplus
}
#endif
#endif /* STENCIL_MI355_H */
