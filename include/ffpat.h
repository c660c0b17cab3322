/*
 * ffpat: one-step full-field photoacoustic reconstruction on AMD MI355X (gfx950).
 *
 * C ABI of libffpat.so.  Method: Haltmeier, Zangerl, Nuster, Nguyen,
 * "Photoacoustic image reconstruction from full field data in heterogeneous
 * media" (2019).  The library applies the forward operator
 *     A = X W_T        (Problem 1, eq. fm; W_T from eq. Wo, X from eq. Radon)
 * its Euclidean transpose A^T = W_T^T X^T (Sec. 3.1), the ramp preconditioner
 * Lambda (Sec. 3.1) and Algorithm 8 (Sec. 3.2), all on the GPU.
 *
 * Discretisation (identical in every entry point):
 *   volumes   [nz][ny][nx], x fastest, contiguous, node-centred:
 *             x_i = (i - (nx-1)/2) dx, y_k = (k - (ny-1)/2) dx, z likewise.
 *             The projection axis is the grid's z axis through its centre.
 *   data      [n_angles][nz][ns], s fastest; detector bin j sits at
 *             s_j = (j - (ns-1)/2) ds on the row of plane z.
 *   angles    phi_a in radians; direction theta = (cos phi, sin phi, 0);
 *             s = x cos phi + y sin phi; rays run along theta-perp.
 *   W_T       leapfrog with dt = T / n_t, n_t = ceil(T c_max / (cfl dx)
 *             (1 - 1e-12)); fourth-order 13-point Laplacian (9-point in 2D
 *             mode) with zero values outside the grid; zero initial
 *             velocity through the symmetric first step
 *             p1 = p0 + (1/2)(c dt)^2 L p0.
 *   X         ray sums with linear interpolation along the minor axis
 *             (weight (dx/m) max(0, 1 - |s_j - t|/(m dx)), m = max(|cos|,|sin|)).
 *   Lambda    Ram-Lak Toeplitz filter along s (taps 1/4, -1/(pi n)^2 for odd
 *             n, 0 for even n), times pi / (n_angles dx^2).
 *
 * Device buffers are caller-owned (`*_dev`, e.g. torch tensor storage),
 * contiguous, of the plan's precision (float or double), on the plan's
 * device.  Every call enqueues on `stream` (a hipStream_t; NULL = the null
 * stream) and returns before the work finishes unless stated otherwise;
 * buffers must stay alive until the stream has passed the call.
 *
 * Errors: every function returns an ffpat_status, never throws or aborts.
 * Argument errors are reported before anything is enqueued.  HIP runtime
 * failures map to FFPAT_EHIP.  ffpat_last_error() gives a thread-local text
 * for the last failure.  A plan is not thread-safe; distinct plans may be
 * used concurrently on distinct streams.  Every call on a plan uses the
 * plan's workspace: calls on one plan enqueued on different streams must be
 * ordered by the caller (events), or they race on the device.
 */
#ifndef FFPAT_H
#define FFPAT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  FFPAT_OK = 0,
  FFPAT_EINVAL = -1,     /* bad argument (null pointer, size, non-finite or non-positive value) */
  FFPAT_ECFL = -2,       /* cfl outside (0, 1/2) in 3D or (0, sqrt(3/8)) in 2D mode: leapfrog unstable */
  FFPAT_ENOMEM = -3,     /* device allocation failed */
  FFPAT_EHIP = -4,       /* HIP runtime error (text in ffpat_last_error) */
  FFPAT_EDIVERGED = -5,  /* non-finite objective or norm during reconstruction */
  FFPAT_EDTYPE = -6,     /* unknown precision */
  FFPAT_EBUSY = -7       /* reserved (not returned by this version) */
} ffpat_status;

typedef enum { FFPAT_F32 = 0, FFPAT_F64 = 1 } ffpat_dtype;

typedef struct ffpat_plan ffpat_plan;  /* opaque */

/* Problem geometry (Problem 1, Sec. 2.1).  All values are read during
 * ffpat_plan_create / ffpat_workspace_bytes only; the plan keeps copies. */
typedef struct {
  int32_t nx, ny, nz;     /* grid nodes; volumes [nz][ny][nx] */
  int32_t ndim;           /* 3 (default, 0 means 3) or 2: z-invariant mode of Sec. 4, Laplacian over x, y */
  double dx;              /* isotropic grid spacing, > 0 */
  double T;               /* measurement time T > 0 (eq. Wo) */
  double cfl;             /* target c_max dt / dx; 0 selects 0.3 */
  int32_t n_angles;       /* >= 1 */
  const double *angles;   /* host array of n_angles radians */
  int32_t ns;             /* detector bins per row; 0 selects nx */
  double ds;              /* detector spacing; 0 selects dx */
  int32_t dtype;          /* ffpat_dtype of every field; reductions are always FP64 */
  uint32_t flags;         /* FFPAT_PLAN_*; other bits: EINVAL */
} ffpat_geom;

/* Plan flags */
#define FFPAT_PLAN_NAIVE_STENCIL 1u   /* unblocked stencil kernel (for comparison) */
#define FFPAT_PLAN_NO_GRAPHS 2u       /* launch every kernel eagerly instead of replaying captured graphs */
#define FFPAT_PLAN_SINGLE_STEP 4u     /* one leapfrog step per stencil pass (no temporal blocking) */
#define FFPAT_PLAN_TWO_STEP 8u        /* at most two leapfrog steps per stencil pass, two wherever the
                                         chain allows */
#define FFPAT_PLAN_THREE_STEP 32u     /* three leapfrog steps per stencil pass wherever the chain and the
                                         grid allow (3D; FP32 with even nx where the 128 x 16 tile is
                                         chosen, FP64), two otherwise.
                                         With none of these three flags the plan chooses, by measurement:
                                         one step per pass below 128^3 voxels; from 128^3 on two, or in
                                         FP32 three where the three-step kernel applies.  More than one:
                                         EINVAL.  Planes of 2^31 bytes or more always take one step per
                                         pass. */

/* Reconstruction flags (ffpat_fb_params.flags) */
#define FFPAT_POSITIVITY 1u   /* R includes the indicator of h >= 0 (prox clamps at 0) */
#define FFPAT_PRECOND    2u   /* data term 1/2 <Lambda r, r> (else 1/2 ||r||^2) */
#define FFPAT_REG_GRAD   4u   /* R = 1/2 ||D h||^2 (forward differences, zero outside) instead of 1/2 ||h||^2 */
#define FFPAT_USE_PLAN_STEP 8u /* reuse the step stored in the plan by an earlier call */
#define FFPAT_TWO_STEP  16u   /* Algorithm 9 (Sec. 4.1): G_dev is the volume g = X^-1 G (see ffpat_fbp),
                                 the data term is 1/2 ||W_T h - g||^2; det_mask must be NULL */

/* Algorithm 8 parameters (Sec. 3.2). */
typedef struct {
  double lambda;            /* regularisation weight >= 0 */
  double step;              /* > 0: constant step s; <= 0: s = 1/L from n_power power-iteration steps */
  int32_t n_iter;           /* K >= 0 iterations */
  int32_t n_power;          /* power-iteration steps (0 selects 20) */
  uint32_t flags;           /* FFPAT_POSITIVITY | FFPAT_PRECOND | FFPAT_REG_GRAD | FFPAT_USE_PLAN_STEP |
                               FFPAT_TWO_STEP; REG_GRAD excludes POSITIVITY; other bits: EINVAL */
  const uint8_t *support;   /* device [nz][ny][nx] mask chi_V (nonzero = inside), or NULL */
  const uint8_t *det_mask;  /* device [n_angles][nz][ns] mask chi_M (nonzero = measured), or NULL */
  double *objective;        /* host array of n_iter values J_k = 1/2<Lambda r_k, r_k> + lambda R(h_k), or NULL */
  double cg_tol;            /* FFPAT_REG_GRAD prox (I + s lambda N)^-1, N = D^T D: with cg_tol and cg_maxit
                               both 0 a 3D grid of at least nx^2 + ny^2 + nz^2 + nx + ny + nz points solves
                               it directly (sine transforms along each axis diagonalise N); otherwise, and in
                               2D mode, by conjugate gradients to this relative residual (0 selects 1e-12 for
                               FP64 plans, 1e-6 for FP32) */
  int32_t cg_maxit;         /* FFPAT_REG_GRAD prox by conjugate gradients: iterations per prox (0 selects
                               200); iterations after convergence are skipped on the device */
} ffpat_fb_params;

/* Library version string. */
const char *ffpat_version(void);

/* Text of the last failure on the calling thread ("" if none). */
const char *ffpat_last_error(void);

/* Device bytes a plan for `geom` allocates (for admission by HBM footprint). */
int ffpat_workspace_bytes(const ffpat_geom *geom, size_t *bytes);

/* Creates a plan on the current device.  c_dev: sound speed c(x) > 0
 * (eq. wave1), [nz][ny][nx] of the plan's precision; it is copied (as
 * (c dt)^2 / (12 dx^2)) and may be freed once `stream` has passed the call.
 * Reads c_max back to the host: this call synchronises `stream`.
 * Returns FFPAT_EINVAL for non-finite or non-positive c. */
int ffpat_plan_create(const ffpat_geom *geom, const void *c_dev, void *stream, ffpat_plan **out);

/* Time grid of the plan: n_t, dt, c_max.  Any pointer may be NULL. */
int ffpat_plan_info(const ffpat_plan *plan, int32_t *nt, double *dt, double *cmax);

/* Leapfrog steps per stencil pass that the plan's wave solves use (eq. leapfrog):
 * 3 or 2 when a temporally blocked kernel runs (see FFPAT_PLAN_THREE_STEP), else 1.
 * A W_T solve is one first-step pass, then passes of that many steps, then a
 * shorter pass for the remainder (the adjoint's last step, which divides by k',
 * always alone). */
int ffpat_plan_steps_per_pass(const ffpat_plan *plan, int32_t *steps);

/* Launch shape of the plan's leapfrog stencil kernel (informational; the kernel
 * that ffpat_plan_steps_per_pass names): tile width and height in grid points and
 * z-planes per work-group.  Chosen per grid, element size and the device the plan
 * was created on (compute units, work-groups a unit holds at once).  0 for all three
 * with FFPAT_PLAN_NAIVE_STENCIL (no tiles).  Any pointer may be NULL. */
int ffpat_plan_stencil_shape(const ffpat_plan *plan, int32_t *tile_x, int32_t *tile_y, int32_t *zchunk);

/* Replaces the plan's sound speed c(x) (eq. wave1) for a new problem of the same
 * geometry, without new allocations: recomputes c_max, n_t, dt and k' from c_dev
 * (as ffpat_plan_create; reads c_max back, so it synchronises `stream`) and discards
 * the stored step size.  Waits for the plan's earlier work (see ffpat_plan_destroy)
 * before touching k'.  Captured graphs are kept when n_t is unchanged (they read k'
 * from the plan's memory) and re-captured at the next use otherwise.  On error
 * (FFPAT_EINVAL for non-finite or non-positive c) the plan keeps its previous
 * speed and time grid. */
int ffpat_plan_set_speed(ffpat_plan *plan, const void *c_dev, void *stream);

/* Releases the plan and its device memory.  Waits for the work of the plan's own
 * calls (an event recorded after each call's work on its stream), not for the
 * rest of the device; work that a caller recorded into a graph of its own must
 * have completed. */
int ffpat_plan_destroy(ffpat_plan *plan);

/* g = X W_T h (Problem 1 with full data; eq. Wo then eq. Radon).
 * h_dev: volume; g_dev: data; must not overlap. */
int ffpat_forward(ffpat_plan *plan, const void *h_dev, void *g_dev, void *stream);

/* h = W_T^T X^T g, the Euclidean transpose of ffpat_forward (Sec. 3.1:
 * backprojection, then the time-reversed wave solve; the transpose of the
 * discrete scheme is (c dt)^-2 W_T((c dt)^2 .)). */
int ffpat_adjoint(ffpat_plan *plan, const void *g_dev, void *h_dev, void *stream);

/* p = W_T h (eq. Wo) alone.  Volumes; must not overlap. */
int ffpat_wave(ffpat_plan *plan, const void *h_dev, void *p_dev, void *stream);

/* q = W_T^T g alone (Euclidean transpose of ffpat_wave). */
int ffpat_wave_adjoint(ffpat_plan *plan, const void *g_dev, void *q_dev, void *stream);

/* g = X v alone (eq. Radon per plane z). */
int ffpat_project(ffpat_plan *plan, const void *vol_dev, void *g_dev, void *stream);

/* v = X^T g alone (backprojection, Sec. 3.1; exact transpose of ffpat_project). */
int ffpat_backproject(ffpat_plan *plan, const void *g_dev, void *vol_dev, void *stream);

/* y = Lambda r alone (Sec. 3.1).  Data arrays; y may equal r (in place). */
int ffpat_ramp(ffpat_plan *plan, const void *r_dev, void *y_dev, void *stream);

/* vol = X^-1 G = X^* Lambda G, filtered backprojection per plane (Sec. 3.1):
 * the first stage of the two-step method (Algorithm 9). */
int ffpat_fbp(ffpat_plan *plan, const void *G_dev, void *vol_dev, void *stream);

/* Algorithm 8 (Sec. 3.2): h_{k+1} = prox_{s lambda R}(h_k - s A^T chi_M Lambda chi_M (A h_k - G)).
 * G_dev: data; h_dev: in h_0 (zeros reproduce the paper's start), out h_K.
 * step_used (host, may be NULL) receives s.  Synchronises `stream` at the
 * end to report the step, the objective values and divergence
 * (FFPAT_EDIVERGED when an objective value or norm is not finite). */
int ffpat_reconstruct(ffpat_plan *plan, const void *G_dev, const ffpat_fb_params *params,
                      void *h_dev, double *step_used, void *stream);

/* Asynchronous form of ffpat_reconstruct for serving loops: enqueues the step
 * selection and params->n_iter iterations on `stream` and returns without any
 * host synchronisation (params->objective is ignored; the values stay on the
 * device).  The power iteration and one FB iteration are captured once as HIP
 * graphs and replayed (unless the plan was created with FFPAT_PLAN_NO_GRAPHS);
 * a change of G_dev, h_dev, masks, flags or lambda re-captures.  Buffers must
 * stay alive until the stream has passed the work. */
int ffpat_fb_enqueue(ffpat_plan *plan, const void *G_dev, const ffpat_fb_params *params, void *h_dev,
                     void *stream);

/* For callers that cannot allocate device memory while they run: code under HIP
 * graph capture, tight serving loops, harnesses that forbid allocation.  The same
 * work as ffpat_fb_enqueue on a plan created beforehand, but it allocates nothing
 * (no hipMalloc or hipFree, no graph or stream of its own): every kernel is launched
 * on `stream` directly, so a caller may record the whole sequence into a graph of its
 * own, and the objective values J_k go to a static device array of the library
 * (65536 FP64 values, 512 KiB per device, held until the process ends) instead of the
 * plan's objective buffer.  params->n_iter above 65536: FFPAT_EINVAL before anything
 * is enqueued; other arguments as ffpat_fb_enqueue.  ffpat_fb_report on the same plan
 * completes the run and reads the values from that array.  Every call on a device
 * shares the array, which keeps the last call's values: calls that overlap on one
 * device (any plans, any streams) race, and a report must come before the next such
 * call on the device. */
int ffpat_fb_enqueue_noalloc(ffpat_plan *plan, const void *G_dev, const ffpat_fb_params *params, void *h_dev,
                             void *stream);

/* Completes an ffpat_fb_enqueue: synchronises `stream`, writes the step size
 * (step_used, may be NULL) and the first n objective values of the last
 * enqueued run (objective, host, may be NULL when n = 0), and returns
 * FFPAT_EDIVERGED if any objective value, norm or the step was not finite. */
int ffpat_fb_report(ffpat_plan *plan, double *step_used, double *objective, int32_t n, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* FFPAT_H */
