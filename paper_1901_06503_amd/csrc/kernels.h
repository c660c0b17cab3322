// Kernel launchers of libffpat (gfx950).  Device code lives in kernels_*.hip;
// the plan and the C ABI (plan.hip) call only these launchers.
#pragma once

#include <hip/hip_runtime.h>
#include <cstddef>
#include <cstdint>

namespace ffpat {

// Grid extents and strides shared by the volume kernels.
struct Dims {
  int nx, ny, nz;
  int ndim;  // 3, or 2 for the z-invariant mode (no z coupling in the Laplacian)
  __host__ __device__ size_t nvox() const { return (size_t)nx * ny * nz; }
};

// Per-angle parameters, computed on the host in double precision.
//
// Projector (Joseph form of the footprint): the ray of bin j crosses marched
// line r (a row y_r if !major_x, a column x_r if major_x) at index position
//     u = u0 + j * uj + r * ur
// along the other axis; the ray sum is w * sum_r lerp(line_r, u), w = dx / m.
//
// Backprojector: voxel (i, k) projects to bin position t = b0 + i * bi + k * bk;
// bin j receives weight w * max(0, 1 - |j - t| * inv_hw), hw = m dx / ds bins.
//
// The FP32 kernels step positions in exact 32.32 fixed point (increments are
// integers, so no rounding accumulates along a ray): ur_fix = ur * 2^32 and
// the backprojector's b0/bi/bk likewise, in bins.
struct AngleParams {
  double u0, uj, ur;
  double b0, bi, bk;
  double hw, inv_hw;
  double w;
  long long ur_fix, b0_fix, bi_fix, bk_fix;
  float inv_hw_f, w_f;   // inv_hw and w rounded to FP32 (the FP32 backprojector's weights)
  int major_x;
  int pad_;
};

// Zero-padded copies read by the projector (line pads) and the backprojector
// (detector-row pads); the pads are zeroed once and never written again.
constexpr int kLinePadL = 3, kLinePadR = 3;   // projector lines: [3 zeros | nm values | 3 zeros]
constexpr int kRowPadL = 2, kRowPadR = 3;     // detector rows:   [2 zeros | ns values | 3 zeros]

enum StepMode : int {
  STEP_FIRST = 0,       // out = p + 1/2 k' S(p)
  STEP_LEAP = 1,        // out = 2 p - prev + k' S(p)      (out may alias prev)
  STEP_FIRST_DIV = 2,   // out = (p + 1/2 k' S(p)) / k'
  STEP_LEAP_DIV = 3     // out = (2 p - prev + k' S(p)) / k'
};

enum StencilKind : int { STENCIL_BLOCKED = 0, STENCIL_NAIVE = 1 };

// One leapfrog step; k' = (c dt)^2 / (12 dx^2); S = integer 13-point (9-point
// in 2D) fourth-order stencil with zero values outside the grid.
template <typename T>
hipError_t launch_wave_step(StencilKind kind, StepMode mode, const Dims &d, const T *p, const T *prev,
                            T *out, const T *kap, hipStream_t s);

// Two leapfrog steps in one pass: q = p(k+1), o = p(k+2) from pm1 = p(k-1), pk = p(k).
// All four buffers must be distinct.
template <typename T>
hipError_t launch_wave_pair(const Dims &d, const T *pm1, const T *pk, T *q, T *o, const T *kap, hipStream_t s);
// Tile (width, height) and planes per work-group that launch_wave_pair takes on the
// current device for this grid.
template <typename T>
void wave_pair_shape(const Dims &d, int *tile_x, int *tile_y, int *zchunk);
// Three leapfrog steps in one pass: r = p(k+2), o = p(k+3) from pm1 = p(k-1), pk =
// p(k) (p(k+1) stays on chip).  first: the pass starts the solve from pk = p(0) with
// zero initial velocity (its first step is STEP_FIRST; pm1 is not read) and yields
// p(2), p(3).  The buffers must be distinct.  *taken = false (and nothing launched)
// where the grid, element size or buffer alignment has no three-step kernel; the
// caller then takes smaller passes.
template <typename T>
hipError_t launch_wave_triple(const Dims &d, const T *pm1, const T *pk, T *r, T *o, const T *kap, hipStream_t s,
                              bool first, bool *taken);
// The first two steps of a solve in one pass: q = p(1), o = p(2) from pk = p(0) with
// zero initial velocity (STEP_FIRST, then STEP_LEAP).  Only where the two-step pass
// runs in wave_step2_split; *taken = false (nothing launched) otherwise.
template <typename T>
hipError_t launch_wave_pair_first(const Dims &d, const T *pk, T *q, T *o, const T *kap, hipStream_t s, bool *taken);
// Three leapfrog steps in one pass whose third is divided by k' (the adjoint solve's
// last three steps): r = p(k+2), o = p(k+3) / k'.  FP32 where launch_wave_triple runs
// wave_step3_wide; *taken = false (nothing launched) otherwise.
template <typename T>
hipError_t launch_wave_triple_div(const Dims &d, const T *pm1, const T *pk, T *r, T *o, const T *kap, hipStream_t s,
                                  bool *taken);
// Two leapfrog steps in one pass whose second is divided by k' (the adjoint solve's
// last two steps, STEP_LEAP then STEP_LEAP_DIV): q = p(k+1), o = p(k+2) / k'.  Only
// where the two-step pass runs in wave_step2_split; *taken = false otherwise.
template <typename T>
hipError_t launch_wave_pair_div(const Dims &d, const T *pm1, const T *pk, T *q, T *o, const T *kap, hipStream_t s,
                                bool *taken);
// Tile and planes per work-group of launch_wave_triple for this grid (8-byte aligned
// buffers); false where it takes no three-step pass.
template <typename T>
bool wave_triple_shape(const Dims &d, int *tile_x, int *tile_y, int *zchunk);
// The same for the one-step blocked kernel (launch_wave_step with STENCIL_BLOCKED).
void wave_step_shape(const Dims &d, size_t esz, int *tile_x, int *tile_y, int *zchunk);
// Whether the two-step kernel is the faster choice for this grid and element size
// (FFPAT_STENCIL_TB=0/1 in the environment overrides the rule).
bool wave_pairs_preferred(const Dims &d, size_t esz);
// Whether a three-step pass exists for this grid and element size (8-byte aligned
// buffers), and whether it is the preferred choice (FFPAT_STENCIL3=0/1 in the
// environment overrides the rule).
template <typename T>
bool wave_triples_available(const Dims &d);
bool wave_triples_preferred(const Dims &d, size_t esz);
// Whether the two-step kernel can address a plane of this grid (plane bytes < 2^31).
bool wave_pairs_fit(const Dims &d, size_t esz);

// k' = (c dt)^2 / (12 dx^2) from c, and c range / finiteness into stats[0..2]
// (min, max, count of non-finite or non-positive values) via block partials.
template <typename T>
hipError_t launch_make_kappa(const Dims &d, const T *c, double dt, double dx, T *kap, hipStream_t s);
template <typename T>
hipError_t launch_c_stats(const Dims &d, const T *c, double *partials, int nblocks, double *stats, hipStream_t s);

// g[a][z][j] = X vol (Joseph ray march).  padN [nz][ny][nx + 6] and padT
// [nz][nx][ny + 6] receive zero-padded copies of vol's rows and of its x-y
// transpose (rays running along x read the transpose); need_n / need_t say
// which copies the angle set uses.  aorder lists the angles that march rows
// (the first n_row_angles entries), then those that march columns.
template <typename T>
hipError_t launch_project(const Dims &d, int n_angles, int ns, const AngleParams *ap, const int *aorder,
                          int n_row_angles, const T *vol, T *padN, T *padT, bool need_n, bool need_t, T *g,
                          hipStream_t s);

// vol = X^T g from detector rows in padded layout gpad [rows][ns + 5]
// (values at offset 2), optionally multiplied point-wise by kap.
// two_tap: every angle's footprint half-width m dx / ds is <= 1 bin.
template <typename T>
hipError_t launch_backproject(const Dims &d, int n_angles, int ns, const AngleParams *ap, bool two_tap,
                              const T *gpad, T *vol, const T *kap, hipStream_t s);

// Copies rows [rows][ns] into the padded row layout (interior only).
template <typename T>
hipError_t launch_pad_rows(int rows, int ns, const T *g, T *gpad, hipStream_t s);

// r = mask * (g - G) (G may be null, mask may be null); y = mask * Lambda r (or
// y = r when taps == nullptr), written at y[row * y_stride + y_off + j].  y may
// alias g (same layout).  row_partials[row] = sum_j r_j y_j when non-null.
template <typename T>
hipError_t launch_residual_ramp(int rows, int ns, const T *g, const T *G, const uint8_t *mask, const T *taps,
                                T *y, int y_stride, int y_off, double *row_partials, hipStream_t s);

// Reductions and element-wise updates (FP64 partials, fixed order).
constexpr int kReduceBlocks = 1024;
constexpr int kReduceThreads = 256;

template <typename T>
hipError_t launch_sumsq(const T *x, size_t n, double *partials, hipStream_t s);  // kReduceBlocks partials
template <typename T>
hipError_t launch_dot(const T *x, const T *y, size_t n, double *partials, hipStream_t s);

// out[0] = scale * sum(partials[0..n)) (single block, fixed order).
hipError_t launch_reduce_to(const double *partials, int n, double scale, double *out, hipStream_t s);

// obj[k] = 0.5 * data + lambda * 0.5 * reg with k = *counter (then *counter += 1;
// values beyond `capacity` are counted but not stored); flags non-finite values.
hipError_t launch_objective(const double *data_sum, const double *reg_sum, double lambda, double *obj,
                            double *counter, int capacity, double *nonfinite_flag, hipStream_t s);

// L = sqrt(sumsq); step = 1 / L.
hipError_t launch_power_finish(const double *sumsq, double *L, double *step, double *nonfinite_flag,
                               hipStream_t s);

template <typename T>
hipError_t launch_fill(T *x, size_t n, double value, hipStream_t s);
// y = x / sqrt(*sumsq)
template <typename T>
hipError_t launch_normalize(const T *x, T *y, size_t n, const double *sumsq, hipStream_t s);

// h <- prox_{s lambda R}(h - s grad) for R = 1/2||h||^2 (+ positivity), support mask.
template <typename T>
hipError_t launch_prox_l2(T *h, const T *grad, size_t n, const double *step, double lambda, int positivity,
                          const uint8_t *support, hipStream_t s);

// f = h - s * grad (gradient regulariser path; prox applied afterwards).
template <typename T>
hipError_t launch_grad_step(const T *h, const T *grad, T *f, size_t n, const double *step, hipStream_t s);

// y = x.
template <typename T>
hipError_t launch_copy(const T *x, T *y, size_t n, hipStream_t s);

}  // namespace ffpat

namespace ffpat {
// y = x * k point-wise (k = k' for the conjugated transpose of W).
template <typename T>
hipError_t launch_mul(const T *x, const T *k, T *y, size_t n, hipStream_t s);
// dst[0] = v (a kernel, so that the write can sit inside a captured graph).
hipError_t launch_set(double *dst, double v, hipStream_t s);
}  // namespace ffpat

namespace ffpat {
// ---- gradient regulariser R = 1/2 ||D h||^2 (D: forward differences / dx, zero
// outside the grid), D^T D = N = -(7-point Laplacian) (5-point in 2D mode).
// partials[b] = sum over block b of h . (N h)
template <typename T>
hipError_t launch_neglap_dot(const Dims &d, double dx, const T *h, double *partials, hipStream_t s);

// Conjugate gradients for (I + tau N) x = f, tau = step[0] * lambda, with FP64
// scalars cg[] on the device: cg[0] rr, cg[1] ff, cg[2] pq, cg[3] rr_new,
// cg[4] alpha, cg[5] beta, cg[6] done flag, cg[7] iterations.
// Every kernel returns at once when cg[6] is set.
template <typename T>
hipError_t launch_cg_init(const Dims &d, double dx, const T *f, const T *x, T *r, T *p, const double *step,
                          double lambda, double *partials_rr, double *partials_ff, hipStream_t s);
template <typename T>
hipError_t launch_cg_apply(const Dims &d, double dx, const T *p, T *q, const double *step, double lambda,
                           const double *cg, double *partials, hipStream_t s);
template <typename T>
hipError_t launch_cg_update(const Dims &d, T *x, T *r, const T *p, const T *q, const double *cg,
                            double *partials, hipStream_t s);
template <typename T>
hipError_t launch_cg_direction(const Dims &d, T *p, const T *r, const double *cg, hipStream_t s);
// Direct prox of the gradient regulariser (3D): sine-transform tables (S_x, S_y, S_z
// row-major, then the eigenvalues mu_x, mu_y, mu_z) into `tab` (at least nx^2 + ny^2 +
// nz^2 + nx + ny + nz elements), one transform along `axis` (0 x, 1 y, 2 z), the scaling.
template <typename T>
hipError_t launch_dst_tables(const Dims &d, double dx, T *tab, hipStream_t s);
template <typename T>
hipError_t launch_dst_axis(const Dims &d, int axis, const T *in, T *out, const T *S, hipStream_t s);
template <typename T>
hipError_t launch_dst_scale(const Dims &d, T *u, const T *mu, const double *step, double lambda, hipStream_t s);
// scalar steps: after init (done if rr <= tol^2 ff), alpha = rr / pq, then beta / convergence
hipError_t launch_cg_check_init(double *cg, double tol, hipStream_t s);
hipError_t launch_cg_alpha(double *cg, hipStream_t s);
hipError_t launch_cg_beta(double *cg, double tol, hipStream_t s);

// h = 0 where support == 0
template <typename T>
hipError_t launch_apply_support(T *h, const uint8_t *support, size_t n, hipStream_t s);
// f = h - step * grad (in place into grad allowed)
// r = w - g (written over w), partials = sum r^2 per block
template <typename T>
hipError_t launch_vol_residual(T *w, const T *g, size_t n, double *partials, hipStream_t s);
}  // namespace ffpat
