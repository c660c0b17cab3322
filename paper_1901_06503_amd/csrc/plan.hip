// Plan, operator composition, Algorithm 8 driver and the C ABI of libffpat.
//
// Operators (Haltmeier, Zangerl, Nuster, Nguyen 2019):
//   W_T       initial-to-final-time wave operator (eq. Wo): n_t leapfrog steps
//   W_T^T     Euclidean transpose: the scheme is a polynomial in K L
//             (K = diag((c dt)^2)), so W_T^T = K^-1 W_T K; the same stepper
//             runs on k' g and the last step divides by k' (Sec. 3.1: the
//             adjoint is a wave solve started from the data at time T)
//   X, X^T    plane-wise X-ray transform (eq. Radon) and backprojection
//   Lambda    ramp filter along s (Sec. 3.1)
//   A = X W_T, A^T = W_T^T X^T
//   Alg. 8    h <- prox_{s lambda R}(h - s A^T chi Lambda chi (A h - G))
//
// Workspace per plan (all device, one allocation): k', four volumes, one
// data array, Ram-Lak taps, per-angle parameters, FP64 partials and scalars.
// No host synchronisation inside the operators or the iteration; device
// scalars (step, L, norms, objective) stay on the device until the end.
#include "kernels.h"
#include "../../include/ffpat.h"

#include <rocprofiler-sdk-roctx/roctx.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

// A named host-side range for timeline tools (roctx; rocprofv3 --marker-trace shows
// them): each C-ABI call that enqueues device work opens one, and the reconstruction
// marks its power iteration, graph captures and FB iterations.  The ranges time the
// host's enqueueing, not the kernels (which the kernel trace shows); without a tool
// attached they cost a call each.
struct TraceRange {
  explicit TraceRange(const char *name) { roctxRangePushA(name); }
  ~TraceRange() { roctxRangePop(); }
  TraceRange(const TraceRange &) = delete;
  TraceRange &operator=(const TraceRange &) = delete;
};

using namespace ffpat;

// Objective history of ffpat_fb_enqueue_noalloc: a static device array, so that entry
// point allocates nothing.  512 KiB per device, held until the process ends; shared by
// every such call on the device (calls that overlap on one device race).
constexpr int kNoAllocMaxIter = 65536;
static __device__ __align__(256) double scratch[kNoAllocMaxIter];

namespace {

thread_local std::string g_last_error;

int fail(int code, const char *fmt, ...)
{
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_last_error = buf;
  return code;
}

int hip_fail(hipError_t e, const char *where)
{
  return fail(FFPAT_EHIP, "%s: %s", where, hipGetErrorString(e));
}

#define HIP_TRY(expr)                                   \
  do {                                                  \
    hipError_t e_ = (expr);                             \
    if (e_ != hipSuccess) return hip_fail(e_, #expr);   \
  } while (0)

// Device scalar slots
enum { SC_STEP = 0, SC_L = 1, SC_REG = 2, SC_DATA = 3, SC_NONFINITE = 4, SC_SUMSQ = 5, SC_ITER = 6, SC_CG = 8,
       SC_COUNT = 16 };   // SC_CG .. SC_CG + 7: conjugate-gradient scalars

constexpr size_t kAlign = 256;
size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

struct DeviceGuard {
  int prev = -1;
  explicit DeviceGuard(int dev)
  {
    if (hipGetDevice(&prev) == hipSuccess && prev != dev) (void)hipSetDevice(dev);
    else prev = -1;
  }
  ~DeviceGuard()
  {
    if (prev >= 0) (void)hipSetDevice(prev);
  }
};

// A captured graph and the arguments it was recorded with.
struct GraphCache {
  hipGraphExec_t exec = nullptr;
  const void *G = nullptr, *h = nullptr, *support = nullptr, *mask = nullptr;
  uint32_t flags = 0;
  double lambda = 0.0, cg_tol = 0.0;
  int n_power = 0, cg_maxit = 0;
  bool matches(const void *G_, const void *h_, const void *sup_, const void *m_, uint32_t f_, double lam_,
               int np_, double tol_, int maxit_) const
  {
    return exec && G == G_ && h == h_ && support == sup_ && mask == m_ && flags == f_ && lambda == lam_ &&
           n_power == np_ && cg_tol == tol_ && cg_maxit == maxit_;
  }
  void set(const void *G_, const void *h_, const void *sup_, const void *m_, uint32_t f_, double lam_, int np_,
           double tol_, int maxit_)
  {
    G = G_; h = h_; support = sup_; mask = m_; flags = f_; lambda = lam_; n_power = np_; cg_tol = tol_;
    cg_maxit = maxit_;
  }
};

struct Layout {
  size_t kap, vol[6], dat, taps, ap, aorder, partials, scalars;
  size_t padN, padT, padD;              // zero-padded copies for the projector / backprojector
  size_t padN_bytes, padT_bytes, padD_bytes;
  size_t total;
  size_t n_partials;
};

}  // namespace

struct ffpat_plan {
  int device = 0;
  Dims d{};
  int dtype = FFPAT_F32;
  size_t esz = 4;
  int n_angles = 0, ns = 0;
  double dx = 0, ds = 0, T = 0, cfl = 0;
  uint32_t flags = 0;
  int nt = 0;
  double dt = 0, cmax = 0, cmin = 0;
  size_t nvox = 0, ndat = 0;
  int rows = 0;
  StencilKind stencil = STENCIL_BLOCKED;
  Layout lay{};
  unsigned char *base = nullptr;
  double *obj = nullptr;  // objective history (device), capacity obj_cap
  int obj_cap = 0;
  double *run_obj = nullptr;  // where the iterations being enqueued write J_k: obj, or the
  int run_obj_cap = 0;        // static history of ffpat_fb_enqueue_noalloc; read by fb_report
  bool has_step = false;
  bool two_tap = true;    // every footprint half-width m dx / ds <= 1 bin
  bool need_n = false;    // some angle marches rows (reads the padded plane)
  bool need_t = false;    // some angle marches columns (reads the padded transpose)
  int n_row_angles = 0;   // angles that march rows (listed first in aorder)
  bool use_graphs = true; // replay captured graphs for the power iteration and FB iterations
  bool use_pairs = true;  // two leapfrog steps per pass where possible
  bool use_triples = false;  // three steps per pass where possible (implies use_pairs)
  hipStream_t cap_stream = nullptr;
  hipEvent_t done = nullptr;  // recorded after the work of every call (ffpat_plan_destroy waits for it)
  GraphCache g_iter, g_power;

  void *vol(int i) const { return base + lay.vol[i]; }
  void *kap() const { return base + lay.kap; }
  void *dat() const { return base + lay.dat; }
  void *taps() const { return base + lay.taps; }
  void *padN() const { return base + lay.padN; }
  void *padT() const { return base + lay.padT; }
  void *padD() const { return base + lay.padD; }
  AngleParams *ap() const { return reinterpret_cast<AngleParams *>(base + lay.ap); }
  int *aorder() const { return reinterpret_cast<int *>(base + lay.aorder); }
  double *partials() const { return reinterpret_cast<double *>(base + lay.partials); }
  double *scalars() const { return reinterpret_cast<double *>(base + lay.scalars); }
};

namespace {

struct Resolved {
  Dims d;
  int dtype, n_angles, ns;
  double dx, ds, T, cfl;
  uint32_t flags;
};

int resolve(const ffpat_geom *g, Resolved *r)
{
  if (!g) return fail(FFPAT_EINVAL, "geometry is NULL");
  if (g->nx < 1 || g->ny < 1 || g->nz < 1) return fail(FFPAT_EINVAL, "grid sizes must be >= 1");
  if (g->nz > 65535) return fail(FFPAT_EINVAL, "nz must be <= 65535");
  const int ndim = g->ndim == 0 ? 3 : g->ndim;
  if (ndim != 2 && ndim != 3) return fail(FFPAT_EINVAL, "ndim must be 2 or 3");
  if (!(g->dx > 0) || !std::isfinite(g->dx)) return fail(FFPAT_EINVAL, "dx must be finite and > 0");
  if (!(g->T > 0) || !std::isfinite(g->T)) return fail(FFPAT_EINVAL, "T must be finite and > 0");
  const double cfl = g->cfl == 0 ? 0.3 : g->cfl;
  const double cfl_max = ndim == 3 ? 0.5 : std::sqrt(3.0 / 8.0);
  if (!(cfl > 0) || !(cfl < cfl_max))
    return fail(FFPAT_ECFL, "cfl %g outside (0, %g): the leapfrog scheme would be unstable", cfl, cfl_max);
  if (g->n_angles < 1 || g->n_angles > 65535) return fail(FFPAT_EINVAL, "n_angles must be in [1, 65535]");
  if (!g->angles) return fail(FFPAT_EINVAL, "angles is NULL");
  for (int a = 0; a < g->n_angles; ++a)
    if (!std::isfinite(g->angles[a])) return fail(FFPAT_EINVAL, "angle %d is not finite", a);
  const int ns = g->ns == 0 ? g->nx : g->ns;
  if (ns < 1 || ns > 8192) return fail(FFPAT_EINVAL, "ns must be in [1, 8192]");
  const double ds = g->ds == 0 ? g->dx : g->ds;
  if (!(ds > 0) || !std::isfinite(ds)) return fail(FFPAT_EINVAL, "ds must be finite and > 0");
  if (g->dtype != FFPAT_F32 && g->dtype != FFPAT_F64) return fail(FFPAT_EDTYPE, "unknown dtype %d", g->dtype);
  // the projector addresses a padded plane (and its padded transpose) with 32-bit
  // byte offsets from the plane's base
  const size_t esz = g->dtype == FFPAT_F64 ? 8 : 4;
  const size_t pad_plane_n = (size_t)g->ny * (size_t)(g->nx + kLinePadL + kLinePadR) * esz;
  const size_t pad_plane_t = (size_t)g->nx * (size_t)(g->ny + kLinePadL + kLinePadR) * esz;
  if (pad_plane_n >= ((size_t)1 << 32) || pad_plane_t >= ((size_t)1 << 32))
    return fail(FFPAT_EINVAL, "an x-y plane of %d x %d %s values is too large for one projection pass "
                "(padded plane of 2^32 bytes or more)", g->nx, g->ny, esz == 8 ? "FP64" : "FP32");
  const size_t nvox = (size_t)g->nx * g->ny * g->nz;
  const size_t ndat = (size_t)g->n_angles * g->nz * ns;
  if (nvox > ((size_t)1 << 33) || ndat > ((size_t)1 << 33)) return fail(FFPAT_EINVAL, "problem too large");
  // work-group counts of the projector / backprojector grids must fit in int
  if ((size_t)g->n_angles * g->nz * (size_t)((ns + 255) / 256) > (size_t)INT32_MAX - 8 ||
      (size_t)((g->nx + 63) / 64) * ((g->ny + 3) / 4) * g->nz > (size_t)INT32_MAX - 8)
    return fail(FFPAT_EINVAL, "problem too large for one launch");
  r->d = Dims{g->nx, g->ny, g->nz, ndim};
  r->dtype = g->dtype;
  r->n_angles = g->n_angles;
  r->ns = ns;
  r->dx = g->dx;
  r->ds = ds;
  r->T = g->T;
  r->cfl = cfl;
  const uint32_t known = FFPAT_PLAN_NAIVE_STENCIL | FFPAT_PLAN_NO_GRAPHS | FFPAT_PLAN_SINGLE_STEP | FFPAT_PLAN_TWO_STEP |
                         FFPAT_PLAN_THREE_STEP;
  if (g->flags & ~known) return fail(FFPAT_EINVAL, "unknown plan flags 0x%x", (unsigned)(g->flags & ~known));
  {
    const uint32_t steps = g->flags & (FFPAT_PLAN_SINGLE_STEP | FFPAT_PLAN_TWO_STEP | FFPAT_PLAN_THREE_STEP);
    if (steps & (steps - 1))
      return fail(FFPAT_EINVAL, "FFPAT_PLAN_SINGLE_STEP, FFPAT_PLAN_TWO_STEP and FFPAT_PLAN_THREE_STEP exclude each other");
  }
  r->flags = g->flags;
  return FFPAT_OK;
}

Layout layout(const Resolved &r)
{
  Layout L{};
  const size_t esz = r.dtype == FFPAT_F64 ? 8 : 4;
  const size_t nvox = r.d.nvox();
  const size_t ndat = (size_t)r.n_angles * r.d.nz * r.ns;
  const size_t rows = (size_t)r.n_angles * r.d.nz;
  size_t off = 0;
  L.kap = off; off = align_up(off + nvox * esz);
  for (int i = 0; i < 6; ++i) { L.vol[i] = off; off = align_up(off + nvox * esz); }
  L.dat = off; off = align_up(off + ndat * esz);
  L.taps = off; off = align_up(off + (size_t)r.ns * esz);
  L.ap = off; off = align_up(off + (size_t)r.n_angles * sizeof(AngleParams));
  L.aorder = off; off = align_up(off + (size_t)r.n_angles * sizeof(int));
  L.n_partials = rows > (size_t)3 * kReduceBlocks ? rows : (size_t)3 * kReduceBlocks;
  L.partials = off; off = align_up(off + L.n_partials * sizeof(double));
  L.scalars = off; off = align_up(off + SC_COUNT * sizeof(double));
  L.padN_bytes = (size_t)r.d.nz * r.d.ny * (r.d.nx + kLinePadL + kLinePadR) * esz;
  L.padT_bytes = (size_t)r.d.nz * r.d.nx * (r.d.ny + kLinePadL + kLinePadR) * esz;
  L.padD_bytes = rows * (size_t)(r.ns + kRowPadL + kRowPadR) * esz;
  L.padN = off; off = align_up(off + L.padN_bytes);
  L.padT = off; off = align_up(off + L.padT_bytes);
  L.padD = off; off = align_up(off + L.padD_bytes);
  L.total = off;
  return L;
}

// Per-angle geometry in double precision (see AngleParams).
AngleParams angle_params(double phi, const Resolved &r)
{
  AngleParams P{};
  const double ca = std::cos(phi), sa = std::sin(phi);
  const double m = std::fmax(std::fabs(ca), std::fabs(sa));
  const double cx = 0.5 * (r.d.nx - 1), cy = 0.5 * (r.d.ny - 1), cs = 0.5 * (r.ns - 1);
  const double dx = r.dx, ds = r.ds;
  P.w = dx / m;
  P.major_x = std::fabs(sa) > std::fabs(ca) ? 1 : 0;
  if (!P.major_x) {
    // rows y_r; x* = (s_j - y_r sin) / cos, u = x*/dx + cx
    P.uj = ds / (dx * ca);
    P.ur = -sa / ca;
    P.u0 = cx - cs * ds / (dx * ca) + cy * sa / ca;
  } else {
    // columns x_r; y* = (s_j - x_r cos) / sin, u = y*/dx + cy
    P.uj = ds / (dx * sa);
    P.ur = -ca / sa;
    P.u0 = cy - cs * ds / (dx * sa) + cx * ca / sa;
  }
  // bin position of voxel (i, k): t = (x_i cos + y_k sin) / ds + cs
  P.bi = dx * ca / ds;
  P.bk = dx * sa / ds;
  P.b0 = cs - cx * dx * ca / ds - cy * dx * sa / ds;
  P.hw = m * dx / ds;
  P.inv_hw = 1.0 / P.hw;
  P.inv_hw_f = (float)P.inv_hw;
  P.w_f = (float)P.w;
  const double two32 = 4294967296.0;
  P.ur_fix = std::llrint(P.ur * two32);
  P.b0_fix = std::llrint(P.b0 * two32);
  P.bi_fix = std::llrint(P.bi * two32);
  P.bk_fix = std::llrint(P.bk * two32);
  return P;
}

// Ram-Lak taps times pi / (n_angles dx^2): makes X^T Lambda X ~ I (filtered
// backprojection over [0, pi) with the ray-sum weights of X).
template <typename T>
std::vector<T> ramp_taps(const Resolved &r)
{
  const double C = M_PI / ((double)r.n_angles * r.dx * r.dx);
  std::vector<T> t((size_t)r.ns);
  for (int n = 0; n < r.ns; ++n) {
    double h = 0.0;
    if (n == 0) h = 0.25;
    else if (n % 2 == 1) h = -1.0 / (M_PI * M_PI * (double)n * (double)n);
    t[(size_t)n] = (T)(C * h);
  }
  return t;
}

// ------------------------------------------------------------------ operators
// Scratch volumes handed to a wave solve (buffers not holding live data).
template <typename T>
struct Pool {
  T *b[6];
  int n = 0;
  Pool(std::initializer_list<void *> v)
  {
    for (void *x : v) b[n++] = static_cast<T *>(x);
  }
  T *take() { return n > 0 ? b[--n] : nullptr; }
  void give(T *x) { b[n++] = x; }
};

// Leapfrog levels after the first step: pm1 = p(k-1), pk = p(k) (pk always a
// scratch buffer; pm1 may be read-only input), `steps` LEAP updates, the last
// one written to `out` (dividing by k' when div_last).  Pairs of steps run in
// the two-step kernel when the plan allows and enough scratch is free.
template <typename T>
int leapfrog_chain(ffpat_plan *P, const T *pm1, bool pm1_owned, T *pk, int steps, T *out, bool div_last,
                   Pool<T> pool, hipStream_t s)
{
  const T *kap = static_cast<const T *>(P->kap());
  while (steps > 0) {
    // steps that may go into multi-step passes (a dividing last step runs alone)
    const int multi = steps - (div_last ? 1 : 0);
    if (P->use_triples && multi >= 3 && pool.n >= (steps == 3 ? 1 : 2)) {
      T *a = pool.take();
      T *b = (steps == 3) ? out : pool.take();
      bool taken = false;
      HIP_TRY(launch_wave_triple<T>(P->d, pm1, pk, a, b, kap, s, false, &taken));
      if (taken) {
        if (pm1_owned) pool.give(const_cast<T *>(pm1));
        pool.give(pk);
        pm1 = a;
        pm1_owned = true;
        pk = b;
        steps -= 3;
        continue;
      }
      if (b != out) pool.give(b);   // buffers the kernel cannot take (alignment): smaller passes
      pool.give(a);
    }
    if (P->use_triples && div_last && steps == 3 && pool.n >= 1) {
      // the adjoint's last three steps in one pass, the third divided by k'
      T *a = pool.take();
      bool taken = false;
      HIP_TRY(launch_wave_triple_div<T>(P->d, pm1, pk, a, out, kap, s, &taken));
      pool.give(a);
      if (taken) return FFPAT_OK;
    }
    if (P->use_pairs && div_last && steps == 2 && pool.n >= 1) {
      // the adjoint's last two steps in one pass, the second divided by k'
      T *a = pool.take();
      bool taken = false;
      HIP_TRY(launch_wave_pair_div<T>(P->d, pm1, pk, a, out, kap, s, &taken));
      pool.give(a);
      if (taken) return FFPAT_OK;
    }
    const bool pair = P->use_pairs && multi >= 2 && pool.n >= (steps == 2 ? 1 : 2);
    if (pair) {
      T *a = pool.take();
      T *b = (steps == 2) ? out : pool.take();
      HIP_TRY(launch_wave_pair<T>(P->d, pm1, pk, a, b, kap, s));
      if (pm1_owned) pool.give(const_cast<T *>(pm1));
      pool.give(pk);
      pm1 = a;
      pm1_owned = true;
      pk = b;
      steps -= 2;
    } else {
      T *dst = (steps == 1) ? out : (pm1_owned ? const_cast<T *>(pm1) : pool.take());
      if (!dst) return fail(FFPAT_EINVAL, "internal: no scratch volume for the leapfrog");
      const StepMode mode = (steps == 1 && div_last) ? STEP_LEAP_DIV : STEP_LEAP;
      HIP_TRY(launch_wave_step<T>(P->stencil, mode, P->d, pk, pm1, dst, kap, s));
      if (pm1_owned && dst != pm1) pool.give(const_cast<T *>(pm1));
      pm1 = pk;
      pm1_owned = true;
      pk = dst;
      steps -= 1;
    }
  }
  return FFPAT_OK;
}

// The first three steps of a solve from p(0) = in in one three-step pass, when the
// plan runs them and at least `after` steps follow: p(2), p(3) into two volumes of
// the pool (p(3) into `out` when nothing follows).  *done = false: not taken.
template <typename T>
int first_triple(ffpat_plan *P, const T *in, T *out, int after, Pool<T> &pool, T **p2, T **p3, bool *done,
                 hipStream_t s)
{
  *done = false;
  if (!P->use_triples || P->nt - 3 < after || pool.n < (P->nt == 3 ? 1 : 2)) return FFPAT_OK;
  T *a = pool.take();
  T *b = (P->nt == 3) ? out : pool.take();
  HIP_TRY(launch_wave_triple<T>(P->d, nullptr, in, a, b, static_cast<const T *>(P->kap()), s, true, done));
  if (!*done) {
    if (b != out) pool.give(b);
    pool.give(a);
    return FFPAT_OK;
  }
  *p2 = a;
  *p3 = b;
  return FFPAT_OK;
}

// The first two steps of a solve from p(0) = in in one two-step pass, where the plan
// runs two-step passes and at least `after` steps follow: p(1), p(2) into two volumes of
// the pool (p(2) into `out` when nothing follows).  *done = false: not taken.
template <typename T>
int first_pair(ffpat_plan *P, const T *in, T *out, int after, Pool<T> &pool, T **p1, T **p2, bool *done,
               hipStream_t s)
{
  *done = false;
  if (!P->use_pairs || P->nt - 2 < after || pool.n < (P->nt == 2 ? 1 : 2)) return FFPAT_OK;
  T *a = pool.take();
  T *b = (P->nt == 2) ? out : pool.take();
  HIP_TRY(launch_wave_pair_first<T>(P->d, in, a, b, static_cast<const T *>(P->kap()), s, done));
  if (!*done) {
    if (b != out) pool.give(b);
    pool.give(a);
    return FFPAT_OK;
  }
  *p1 = a;
  *p2 = b;
  return FFPAT_OK;
}

// out = W_T in (in read-only; pool: scratch volumes distinct from in and out)
template <typename T>
int wave_forward(ffpat_plan *P, const T *in, T *out, Pool<T> pool, hipStream_t s)
{
  const T *kap = static_cast<const T *>(P->kap());
  if (P->nt == 1) {
    HIP_TRY(launch_wave_step<T>(P->stencil, STEP_FIRST, P->d, in, nullptr, out, kap, s));
    return FFPAT_OK;
  }
  T *p2 = nullptr, *p3 = nullptr;
  bool done = false;
  if (int rc = first_triple<T>(P, in, out, 0, pool, &p2, &p3, &done, s)) return rc;
  if (done) return P->nt == 3 ? FFPAT_OK : leapfrog_chain<T>(P, p2, true, p3, P->nt - 3, out, false, pool, s);
  T *q1 = nullptr, *q2 = nullptr;
  if (int rc = first_pair<T>(P, in, out, 0, pool, &q1, &q2, &done, s)) return rc;
  if (done) return P->nt == 2 ? FFPAT_OK : leapfrog_chain<T>(P, q1, true, q2, P->nt - 2, out, false, pool, s);
  T *p1 = pool.take();
  HIP_TRY(launch_wave_step<T>(P->stencil, STEP_FIRST, P->d, in, nullptr, p1, kap, s));
  return leapfrog_chain<T>(P, in, false, p1, P->nt - 1, out, false, pool, s);
}

// out = K^-1 W_T K g given b = k' g already in `b` (overwritten).
template <typename T>
int wave_adjoint_from_scaled(ffpat_plan *P, T *b, T *out, Pool<T> pool, hipStream_t s)
{
  const T *kap = static_cast<const T *>(P->kap());
  if (P->nt == 1) {
    HIP_TRY(launch_wave_step<T>(P->stencil, STEP_FIRST_DIV, P->d, b, nullptr, out, kap, s));
    return FFPAT_OK;
  }
  // the last step divides by k', so a first three-step pass needs a step after it
  T *p2 = nullptr, *p3 = nullptr;
  bool done = false;
  if (int rc = first_triple<T>(P, b, out, 1, pool, &p2, &p3, &done, s)) return rc;
  if (done) {
    pool.give(b);
    return leapfrog_chain<T>(P, p2, true, p3, P->nt - 3, out, true, pool, s);
  }
  T *q1 = nullptr, *q2 = nullptr;
  if (int rc = first_pair<T>(P, b, out, 1, pool, &q1, &q2, &done, s)) return rc;
  if (done) {
    pool.give(b);
    return leapfrog_chain<T>(P, q1, true, q2, P->nt - 2, out, true, pool, s);
  }
  T *p1 = pool.take();
  HIP_TRY(launch_wave_step<T>(P->stencil, STEP_FIRST, P->d, b, nullptr, p1, kap, s));
  return leapfrog_chain<T>(P, b, true, p1, P->nt - 1, out, true, pool, s);
}

template <typename T>
int wave_adjoint_op(ffpat_plan *P, const T *g, T *q, hipStream_t s)
{
  T *V1 = static_cast<T *>(P->vol(0));
  HIP_TRY(launch_mul<T>(g, static_cast<const T *>(P->kap()), V1, P->nvox, s));
  return wave_adjoint_from_scaled<T>(P, V1, q, Pool<T>{P->vol(1), P->vol(2), P->vol(4)}, s);
}

template <typename T>
hipError_t project(ffpat_plan *P, const T *vol, T *g, hipStream_t s)
{
  return launch_project<T>(P->d, P->n_angles, P->ns, P->ap(), P->aorder(), P->n_row_angles, vol,
                           static_cast<T *>(P->padN()),
                           static_cast<T *>(P->padT()), P->need_n, P->need_t, g, s);
}

template <typename T>
hipError_t backproject_op(ffpat_plan *P, const T *g, T *vol, hipStream_t s)
{
  hipError_t e = launch_pad_rows<T>(P->rows, P->ns, g, static_cast<T *>(P->padD()), s);
  if (e != hipSuccess) return e;
  return launch_backproject<T>(P->d, P->n_angles, P->ns, P->ap(), P->two_tap, static_cast<const T *>(P->padD()),
                               vol, nullptr, s);
}

template <typename T>
int op_forward(ffpat_plan *P, const T *h, T *g, hipStream_t s)
{
  T *V2 = static_cast<T *>(P->vol(1));
  int rc = wave_forward<T>(P, h, V2, Pool<T>{P->vol(0), P->vol(2), P->vol(4), P->vol(5)}, s);
  if (rc) return rc;
  HIP_TRY(project<T>(P, V2, g, s));
  return FFPAT_OK;
}

// h = A^T y for y already in the padded row buffer.
template <typename T>
int op_adjoint_padded(ffpat_plan *P, T *h, hipStream_t s)
{
  T *V1 = static_cast<T *>(P->vol(0));
  HIP_TRY(launch_backproject<T>(P->d, P->n_angles, P->ns, P->ap(), P->two_tap, static_cast<const T *>(P->padD()),
                                V1, static_cast<const T *>(P->kap()), s));
  return wave_adjoint_from_scaled<T>(P, V1, h, Pool<T>{P->vol(1), P->vol(4), P->vol(5)}, s);
}

template <typename T>
int op_adjoint(ffpat_plan *P, const T *g, T *h, hipStream_t s)
{
  HIP_TRY(launch_pad_rows<T>(P->rows, P->ns, g, static_cast<T *>(P->padD()), s));
  return op_adjoint_padded<T>(P, h, s);
}

// y = chi Lambda chi (A v - G) (G may be null), written into the padded row
// buffer that the backprojector reads: the data-space part of one iteration.
template <typename T>
int data_residual(ffpat_plan *P, const T *v, const T *G, const uint8_t *mask, bool precond, double *row_partials,
                  hipStream_t s)
{
  T *D = static_cast<T *>(P->dat());
  int rc = op_forward<T>(P, v, D, s);
  if (rc) return rc;
  HIP_TRY(launch_residual_ramp<T>(P->rows, P->ns, D, G, mask, precond ? static_cast<const T *>(P->taps()) : nullptr,
                                  static_cast<T *>(P->padD()), P->ns + kRowPadL + kRowPadR, kRowPadL, row_partials,
                                  s));
  return FFPAT_OK;
}

// Conjugate-gradient iteration controls (defaults when the caller passes 0).
struct CgControl {
  double tol;
  int maxit;
};

template <typename T>
CgControl cg_control(const ffpat_fb_params *prm)
{
  CgControl c;
  c.tol = prm->cg_tol > 0 ? prm->cg_tol : (sizeof(T) == 8 ? 1e-12 : 1e-6);
  c.maxit = prm->cg_maxit > 0 ? prm->cg_maxit : 200;
  return c;
}

// w = A^T chi Lambda chi A v (one-step) or W^T W v (two-step) into V3; scratch V1, V2.
template <typename T>
int normal_operator(ffpat_plan *P, const T *v, bool two_step, bool precond, const uint8_t *mask, hipStream_t s)
{
  T *V1 = static_cast<T *>(P->vol(0)), *V2 = static_cast<T *>(P->vol(1)), *V3 = static_cast<T *>(P->vol(2));
  if (two_step) {
    int rc = wave_forward<T>(P, v, V2, Pool<T>{P->vol(0), P->vol(2), P->vol(4), P->vol(5)}, s);
    if (rc) return rc;
    HIP_TRY(launch_mul<T>(V2, static_cast<const T *>(P->kap()), V1, P->nvox, s));
    return wave_adjoint_from_scaled<T>(P, V1, V3, Pool<T>{P->vol(1), P->vol(4), P->vol(5)}, s);
  }
  int rc = data_residual<T>(P, v, nullptr, mask, precond, nullptr, s);
  if (rc) return rc;
  return op_adjoint_padded<T>(P, V3, s);
}

template <typename T>
int power_iteration(ffpat_plan *P, int n_power, bool two_step, bool precond, const uint8_t *mask, hipStream_t s)
{
  T *V3 = static_cast<T *>(P->vol(2)), *V4 = static_cast<T *>(P->vol(3));
  double *sc = P->scalars();
  HIP_TRY(launch_fill<T>(V4, P->nvox, 1.0 / std::sqrt((double)P->nvox), s));
  for (int it = 0; it < n_power; ++it) {
    int rc = normal_operator<T>(P, V4, two_step, precond, mask, s);
    if (rc) return rc;
    HIP_TRY(launch_sumsq<T>(V3, P->nvox, P->partials(), s));
    HIP_TRY(launch_reduce_to(P->partials(), kReduceBlocks, 1.0, sc + SC_SUMSQ, s));
    HIP_TRY(launch_normalize<T>(V3, V4, P->nvox, sc + SC_SUMSQ, s));
  }
  HIP_TRY(launch_power_finish(sc + SC_SUMSQ, sc + SC_L, sc + SC_STEP, sc + SC_NONFINITE, s));
  return FFPAT_OK;
}

// Whether the gradient regulariser's prox is solved directly by sine transforms: 3D,
// no conjugate-gradient controls given, and the transform tables fit in a volume.
bool prox_by_sine_transforms(const ffpat_plan *P, const ffpat_fb_params *prm)
{
  const size_t nx = P->d.nx, ny = P->d.ny, nz = P->d.nz;
  return P->d.ndim == 3 && prm->cg_tol <= 0 && prm->cg_maxit <= 0 &&
         nx * nx + ny * ny + nz * nz + nx + ny + nz <= P->nvox;
}

// h <- prox_{s lambda R}(h - s grad), grad in V3.  l2 (+ positivity): closed form;
// gradient regulariser: (I + s lambda N) h = f with f in V1, either directly (three
// sine transforms, the scaling, three transforms; tables in V3, ping-pong through V2
// and V4) or by conjugate gradients started from h_k (r, p, q in V2, V4, V3).
// Support mask applied last.
template <typename T>
int prox_step(ffpat_plan *P, T *h, const ffpat_fb_params *prm, hipStream_t s)
{
  T *V1 = static_cast<T *>(P->vol(0)), *V2 = static_cast<T *>(P->vol(1)), *V3 = static_cast<T *>(P->vol(2)),
    *V4 = static_cast<T *>(P->vol(3));
  double *sc = P->scalars();
  if (!(prm->flags & FFPAT_REG_GRAD)) {
    HIP_TRY(launch_prox_l2<T>(h, V3, P->nvox, sc + SC_STEP, prm->lambda, (prm->flags & FFPAT_POSITIVITY) ? 1 : 0,
                              prm->support, s));
    return FFPAT_OK;
  }
  const CgControl cc = cg_control<T>(prm);
  double *cg = sc + SC_CG;
  double *pa = P->partials(), *pb = P->partials() + kReduceBlocks;
  HIP_TRY(launch_grad_step<T>(h, V3, V1, P->nvox, sc + SC_STEP, s));                 // f = h - s grad
  if (prox_by_sine_transforms(P, prm)) {
    const Dims &d = P->d;
    T *tab = V3;                                                                       // grad is consumed
    const T *Sx = tab, *Sy = Sx + (size_t)d.nx * d.nx, *Sz = Sy + (size_t)d.ny * d.ny;
    const T *mu = Sz + (size_t)d.nz * d.nz;
    HIP_TRY(launch_dst_tables<T>(d, P->dx, tab, s));
    HIP_TRY(launch_dst_axis<T>(d, 0, V1, V2, Sx, s));
    HIP_TRY(launch_dst_axis<T>(d, 1, V2, V4, Sy, s));
    HIP_TRY(launch_dst_axis<T>(d, 2, V4, V2, Sz, s));
    HIP_TRY(launch_dst_scale<T>(d, V2, mu, sc + SC_STEP, prm->lambda, s));
    HIP_TRY(launch_dst_axis<T>(d, 0, V2, V4, Sx, s));
    HIP_TRY(launch_dst_axis<T>(d, 1, V4, V2, Sy, s));
    HIP_TRY(launch_dst_axis<T>(d, 2, V2, h, Sz, s));
    if (prm->support) HIP_TRY(launch_apply_support<T>(h, prm->support, P->nvox, s));
    return FFPAT_OK;
  }
  HIP_TRY(launch_cg_init<T>(P->d, P->dx, V1, h, V2, V4, sc + SC_STEP, prm->lambda, pa, pb, s));
  HIP_TRY(launch_reduce_to(pa, kReduceBlocks, 1.0, cg + 0, s));
  HIP_TRY(launch_reduce_to(pb, kReduceBlocks, 1.0, cg + 1, s));
  HIP_TRY(launch_cg_check_init(cg, cc.tol, s));
  for (int it = 0; it < cc.maxit; ++it) {
    HIP_TRY(launch_cg_apply<T>(P->d, P->dx, V4, V3, sc + SC_STEP, prm->lambda, cg, pa, s));
    HIP_TRY(launch_reduce_to(pa, kReduceBlocks, 1.0, cg + 2, s));
    HIP_TRY(launch_cg_alpha(cg, s));
    HIP_TRY(launch_cg_update<T>(P->d, h, V2, V4, V3, cg, pa, s));
    HIP_TRY(launch_reduce_to(pa, kReduceBlocks, 1.0, cg + 3, s));
    HIP_TRY(launch_cg_beta(cg, cc.tol, s));
    HIP_TRY(launch_cg_direction<T>(P->d, V4, V2, cg, s));
  }
  if (prm->support) HIP_TRY(launch_apply_support<T>(h, prm->support, P->nvox, s));
  return FFPAT_OK;
}

// One iteration of Algorithm 8 (or of Algorithm 9 with FFPAT_TWO_STEP, where G
// is the volume g = X^-1 G and the operator is W_T).  The objective goes to
// obj[counter], counter++ (device-side), so the same launch sequence serves
// every iteration and can be captured once as a graph.
template <typename T>
int fb_iteration(ffpat_plan *P, const T *G, T *h, const ffpat_fb_params *prm, hipStream_t s)
{
  const bool precond = prm->flags & FFPAT_PRECOND;
  const bool two_step = prm->flags & FFPAT_TWO_STEP;
  T *V1 = static_cast<T *>(P->vol(0)), *V2 = static_cast<T *>(P->vol(1)), *V3 = static_cast<T *>(P->vol(2));
  double *sc = P->scalars();
  // R(h_k) for the objective: ||h||^2 or h . N h
  if (prm->flags & FFPAT_REG_GRAD) HIP_TRY(launch_neglap_dot<T>(P->d, P->dx, h, P->partials(), s));
  else HIP_TRY(launch_sumsq<T>(h, P->nvox, P->partials(), s));
  HIP_TRY(launch_reduce_to(P->partials(), kReduceBlocks, 1.0, sc + SC_REG, s));
  int rc;
  if (two_step) {
    // r = W h - g, data term ||r||^2, gradient W^T r
    rc = wave_forward<T>(P, h, V2, Pool<T>{P->vol(0), P->vol(2), P->vol(4), P->vol(5)}, s);
    if (rc) return rc;
    HIP_TRY(launch_vol_residual<T>(V2, G, P->nvox, P->partials(), s));
    HIP_TRY(launch_reduce_to(P->partials(), kReduceBlocks, 1.0, sc + SC_DATA, s));
    HIP_TRY(launch_objective(sc + SC_DATA, sc + SC_REG, prm->lambda, P->run_obj, sc + SC_ITER, P->run_obj_cap,
                             sc + SC_NONFINITE, s));
    HIP_TRY(launch_mul<T>(V2, static_cast<const T *>(P->kap()), V1, P->nvox, s));
    rc = wave_adjoint_from_scaled<T>(P, V1, V3, Pool<T>{P->vol(1), P->vol(4), P->vol(5)}, s);
    if (rc) return rc;
  } else {
    // r = chi (A h - G), y = chi Lambda r, data term, gradient A^T y
    rc = data_residual<T>(P, h, G, prm->det_mask, precond, P->partials(), s);
    if (rc) return rc;
    HIP_TRY(launch_reduce_to(P->partials(), P->rows, 1.0, sc + SC_DATA, s));
    HIP_TRY(launch_objective(sc + SC_DATA, sc + SC_REG, prm->lambda, P->run_obj, sc + SC_ITER, P->run_obj_cap,
                             sc + SC_NONFINITE, s));
    rc = op_adjoint_padded<T>(P, V3, s);
    if (rc) return rc;
  }
  return prox_step<T>(P, h, prm, s);
}

// Records `body(stream)` into a graph on the plan's capture stream.
template <typename F>
int capture_graph(ffpat_plan *P, GraphCache &gc, F &&body)
{
  TraceRange trace("graph_capture");
  if (!P->cap_stream) HIP_TRY(hipStreamCreateWithFlags(&P->cap_stream, hipStreamNonBlocking));
  if (gc.exec) {
    HIP_TRY(hipGraphExecDestroy(gc.exec));
    gc.exec = nullptr;
  }
  HIP_TRY(hipStreamBeginCapture(P->cap_stream, hipStreamCaptureModeThreadLocal));
  const int rc = body(P->cap_stream);
  hipGraph_t graph = nullptr;
  const hipError_t e = hipStreamEndCapture(P->cap_stream, &graph);
  if (rc) {
    if (e == hipSuccess && graph) (void)hipGraphDestroy(graph);
    return rc;
  }
  if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture");
  hipGraphExec_t exec = nullptr;
  const hipError_t ei = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
  (void)hipGraphDestroy(graph);
  if (ei != hipSuccess) return hip_fail(ei, "hipGraphInstantiate");
  gc.exec = exec;
  return FFPAT_OK;
}

int ensure_objective_capacity(ffpat_plan *P, int n, hipStream_t s)
{
  if (n <= P->obj_cap) return FFPAT_OK;
  const int cap = n > 1024 ? n : 1024;
  // The captured iteration holds the buffer and its capacity as kernel arguments:
  // it is captured again after the buffer moves.
  if (P->g_iter.exec) {
    HIP_TRY(hipStreamSynchronize(s));
    (void)hipGraphExecDestroy(P->g_iter.exec);
    P->g_iter.exec = nullptr;
  }
  if (P->obj) {
    HIP_TRY(hipStreamSynchronize(s));
    HIP_TRY(hipFree(P->obj));
    P->obj = nullptr;
    P->obj_cap = 0;
  }
  const hipError_t e = hipMalloc(&P->obj, sizeof(double) * (size_t)cap);
  if (e != hipSuccess) {
    P->obj = nullptr;
    (void)hipGetLastError();   // handled here: later launch checks must not see it
    return fail(FFPAT_ENOMEM, "hipMalloc of %d objective values failed: %s", cap, hipGetErrorString(e));
  }
  P->obj_cap = cap;
  return FFPAT_OK;
}

// Enqueues the step-size selection and n_iter iterations; no host synchronisation.
// static_obj != nullptr: the objective values go to that device array (capacity
// kNoAllocMaxIter) and every kernel is launched on `s` directly (no graph capture, no
// allocation: the no-allocation entry point).
template <typename T>
int fb_enqueue(ffpat_plan *P, const T *G, const ffpat_fb_params *prm, T *h, hipStream_t s,
               double *static_obj = nullptr)
{
  const bool precond = prm->flags & FFPAT_PRECOND;
  const bool two_step = prm->flags & FFPAT_TWO_STEP;
  const int n_power = prm->n_power > 0 ? prm->n_power : 20;
  const bool graphs = P->use_graphs && !static_obj;
  double *sc = P->scalars();
  if (static_obj) {
    P->run_obj = static_obj;
    P->run_obj_cap = kNoAllocMaxIter;
  } else {
    int rc = ensure_objective_capacity(P, prm->n_iter, s);
    if (rc) return rc;
    P->run_obj = P->obj;
    P->run_obj_cap = P->obj_cap;
  }
  int rc = FFPAT_OK;
  HIP_TRY(launch_set(sc + SC_NONFINITE, 0.0, s));
  HIP_TRY(launch_set(sc + SC_ITER, 0.0, s));
  if (prm->flags & FFPAT_USE_PLAN_STEP) {
    if (!P->has_step) return fail(FFPAT_EINVAL, "FFPAT_USE_PLAN_STEP but the plan holds no step yet");
  } else if (prm->step > 0) {
    HIP_TRY(launch_set(sc + SC_STEP, prm->step, s));
  } else if (graphs) {
    TraceRange trace("power_iteration");
    const uint32_t key = prm->flags & (FFPAT_PRECOND | FFPAT_TWO_STEP);
    if (!P->g_power.matches(nullptr, nullptr, nullptr, prm->det_mask, key, 0.0, n_power, 0.0, 0)) {
      rc = capture_graph(P, P->g_power, [&](hipStream_t cs) {
        return power_iteration<T>(P, n_power, two_step, precond, prm->det_mask, cs);
      });
      if (rc) return rc;
      P->g_power.set(nullptr, nullptr, nullptr, prm->det_mask, key, 0.0, n_power, 0.0, 0);
    }
    HIP_TRY(hipGraphLaunch(P->g_power.exec, s));
  } else {
    TraceRange trace("power_iteration");
    rc = power_iteration<T>(P, n_power, two_step, precond, prm->det_mask, s);
    if (rc) return rc;
  }
  P->has_step = true;
  if (prm->n_iter <= 0) return FFPAT_OK;
  TraceRange trace("fb_iterations");
  if (graphs) {
    const uint32_t key = prm->flags & (FFPAT_PRECOND | FFPAT_POSITIVITY | FFPAT_REG_GRAD | FFPAT_TWO_STEP);
    const CgControl cc = cg_control<T>(prm);
    if (!P->g_iter.matches(G, h, prm->support, prm->det_mask, key, prm->lambda, 0, cc.tol, cc.maxit)) {
      rc = capture_graph(P, P->g_iter, [&](hipStream_t cs) { return fb_iteration<T>(P, G, h, prm, cs); });
      if (rc) return rc;
      P->g_iter.set(G, h, prm->support, prm->det_mask, key, prm->lambda, 0, cc.tol, cc.maxit);
    }
    for (int k = 0; k < prm->n_iter; ++k) HIP_TRY(hipGraphLaunch(P->g_iter.exec, s));
  } else {
    for (int k = 0; k < prm->n_iter; ++k) {
      rc = fb_iteration<T>(P, G, h, prm, s);
      if (rc) return rc;
    }
  }
  return FFPAT_OK;
}

// Waits for `s`, then reports the step, up to n objective values and divergence.
int fb_report(ffpat_plan *P, double *step_used, double *objective, int n, hipStream_t s)
{
  double host_sc[SC_COUNT];
  HIP_TRY(hipMemcpyAsync(host_sc, P->scalars(), sizeof host_sc, hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  const int done = (int)host_sc[SC_ITER];
  if (objective && n > 0) {
    if (n > done || n > P->run_obj_cap || !P->run_obj)
      return fail(FFPAT_EINVAL, "%d objective values requested, %d available", n, done);
    HIP_TRY(hipMemcpyAsync(objective, P->run_obj, sizeof(double) * (size_t)n, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
  }
  if (step_used) *step_used = host_sc[SC_STEP];
  if (host_sc[SC_NONFINITE] != 0.0 || !std::isfinite(host_sc[SC_STEP]))
    return fail(FFPAT_EDIVERGED, "non-finite objective, norm or step during reconstruction");
  return FFPAT_OK;
}

template <typename T>
int reconstruct(ffpat_plan *P, const T *G, const ffpat_fb_params *prm, T *h, double *step_used, hipStream_t s)
{
  int rc = fb_enqueue<T>(P, G, prm, h, s);
  if (rc) return rc;
  return fb_report(P, step_used, prm->objective, prm->objective ? prm->n_iter : 0, s);
}

template <typename T>
int fbp_op(ffpat_plan *P, const T *G, T *vol, hipStream_t s)
{
  HIP_TRY(launch_residual_ramp<T>(P->rows, P->ns, G, nullptr, nullptr, static_cast<const T *>(P->taps()),
                                  static_cast<T *>(P->padD()), P->ns + kRowPadL + kRowPadR, kRowPadL, nullptr, s));
  HIP_TRY(launch_backproject<T>(P->d, P->n_angles, P->ns, P->ap(), P->two_tap, static_cast<const T *>(P->padD()),
                                vol, nullptr, s));
  return FFPAT_OK;
}

bool is_f64(const ffpat_plan *P) { return P->dtype == FFPAT_F64; }

// Records the plan's completion event after a call's work on `s` (when the call
// succeeded): ffpat_plan_destroy and ffpat_plan_set_speed wait for the plan's own
// work only, not for the device.
// Work that a caller records into a graph of its own is not tracked (the caller
// completes its replays before destroying the plan).
int mark_done(ffpat_plan *P, hipStream_t s, int rc)
{
  if (rc != FFPAT_OK) return rc;
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  hipError_t e = hipStreamIsCapturing(s, &cs);
  if (e != hipSuccess) return hip_fail(e, "hipStreamIsCapturing");
  if (cs != hipStreamCaptureStatusNone) return FFPAT_OK;
  e = hipEventRecord(P->done, s);
  return e == hipSuccess ? FFPAT_OK : hip_fail(e, "hipEventRecord");
}

// c range and validity (one host read), the time grid and k' of a plan for sound
// speed c_dev, on stream s.  On error the plan's previous k' and time grid stay.
int apply_speed(ffpat_plan *P, const void *c_dev, hipStream_t s)
{
  double stats[3];
  double *sc = P->scalars();
  hipError_t e;
  if (is_f64(P)) e = launch_c_stats<double>(P->d, static_cast<const double *>(c_dev), P->partials(), kReduceBlocks, sc, s);
  else e = launch_c_stats<float>(P->d, static_cast<const float *>(c_dev), P->partials(), kReduceBlocks, sc, s);
  if (e == hipSuccess) e = hipMemcpyAsync(stats, sc, sizeof stats, hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return hip_fail(e, "sound-speed statistics");
  if (stats[2] != 0.0) return fail(FFPAT_EINVAL, "c has %.0f non-finite or non-positive values", stats[2]);
  // time grid: dt = cfl dx / c_max, rounded so that n_t dt = T exactly
  const double x = P->T * stats[1] / (P->cfl * P->dx);
  double n = std::ceil(x * (1.0 - 1e-12));
  if (n < 1.0) n = 1.0;
  if (n > 1e7) return fail(FFPAT_EINVAL, "n_t = %g time steps is unreasonably large", n);
  P->cmin = stats[0];
  P->cmax = stats[1];
  P->nt = (int)n;
  P->dt = P->T / n;
  if (is_f64(P)) e = launch_make_kappa<double>(P->d, static_cast<const double *>(c_dev), P->dt, P->dx, static_cast<double *>(P->kap()), s);
  else e = launch_make_kappa<float>(P->d, static_cast<const float *>(c_dev), P->dt, P->dx, static_cast<float *>(P->kap()), s);
  if (e != hipSuccess) return hip_fail(e, "make_kappa");
  return FFPAT_OK;
}

// Device address of `scratch` (the objective history of ffpat_fb_enqueue_noalloc) on
// each device, resolved once per device with that device current: every GPU holds its
// own copy of the array at its own address, and in host code the array's name is not
// a device address.
constexpr int kMaxScratchDevices = 64;
std::mutex g_scratch_mu;
double *g_scratch_ptr[kMaxScratchDevices] = {};

// Resolves the address for the current device `dev` if not done yet.
int scratch_resolve(int dev)
{
  if (dev < 0 || dev >= kMaxScratchDevices)
    return fail(FFPAT_EINVAL, "device %d: the static history is kept for devices 0..%d", dev, kMaxScratchDevices - 1);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch_ptr[dev]) return FFPAT_OK;
  void *p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess || !p) {
    (void)hipGetLastError();   // reported here: later launch checks must not see it
    return fail(FFPAT_EHIP, "hipGetSymbolAddress of the static objective history: %s", hipGetErrorString(e));
  }
  g_scratch_ptr[dev] = static_cast<double *>(p);
  return FFPAT_OK;
}

double *scratch_address(int dev)
{
  if (dev < 0 || dev >= kMaxScratchDevices) return nullptr;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  return g_scratch_ptr[dev];
}

#define CHECK_PLAN(P)                                               \
  do {                                                              \
    if (!(P)) return fail(FFPAT_EINVAL, "plan is NULL");            \
  } while (0)
#define CHECK_PTR(p, name)                                          \
  do {                                                              \
    if (!(p)) return fail(FFPAT_EINVAL, "%s is NULL", name);        \
  } while (0)

}  // namespace

// ============================================================================ C ABI
extern "C" {

const char *ffpat_version(void) { return "ffpat 0.1 (gfx950)"; }

const char *ffpat_last_error(void) { return g_last_error.c_str(); }

int ffpat_workspace_bytes(const ffpat_geom *geom, size_t *bytes)
{
  Resolved r;
  int rc = resolve(geom, &r);
  if (rc) return rc;
  CHECK_PTR(bytes, "bytes");
  *bytes = layout(r).total;
  return FFPAT_OK;
}

int ffpat_plan_create(const ffpat_geom *geom, const void *c_dev, void *stream, ffpat_plan **out)
{
  TraceRange trace("ffpat_plan_create");
  CHECK_PTR(out, "out");
  *out = nullptr;
  Resolved r;
  int rc = resolve(geom, &r);
  if (rc) return rc;
  CHECK_PTR(c_dev, "c_dev");
  hipStream_t s = static_cast<hipStream_t>(stream);

  ffpat_plan *P = new (std::nothrow) ffpat_plan();
  if (!P) return fail(FFPAT_ENOMEM, "host allocation failed");
  hipError_t e = hipGetDevice(&P->device);
  if (e != hipSuccess) {
    delete P;
    return hip_fail(e, "hipGetDevice");
  }
  // set-up of the no-allocation entry point on this device (a failure is reported by
  // that entry point, which tries again; plan creation does not depend on it)
  (void)scratch_resolve(P->device);
  P->d = r.d;
  P->dtype = r.dtype;
  P->esz = r.dtype == FFPAT_F64 ? 8 : 4;
  P->n_angles = r.n_angles;
  P->ns = r.ns;
  P->dx = r.dx;
  P->ds = r.ds;
  P->T = r.T;
  P->cfl = r.cfl;
  P->flags = r.flags;
  P->stencil = (r.flags & FFPAT_PLAN_NAIVE_STENCIL) ? STENCIL_NAIVE : STENCIL_BLOCKED;
  P->use_graphs = !(r.flags & FFPAT_PLAN_NO_GRAPHS);
  {
    const size_t esz = r.dtype == FFPAT_F64 ? 8 : 4;
    const bool forced = r.flags & (FFPAT_PLAN_TWO_STEP | FFPAT_PLAN_THREE_STEP);
    const bool triples = esz == 8 ? wave_triples_available<double>(r.d) : wave_triples_available<float>(r.d);
    // three steps per pass where preferred, also on grids small enough for one step
    // per pass otherwise (multi-step passes imply use_pairs, for the remainders)
    const bool triples_preferred = triples && !forced && wave_triples_preferred(r.d, esz);
    P->use_pairs = P->stencil == STENCIL_BLOCKED && wave_pairs_fit(r.d, esz) &&
                   (forced || (!(r.flags & FFPAT_PLAN_SINGLE_STEP) &&
                               (wave_pairs_preferred(r.d, esz) || triples_preferred)));
    P->use_triples = P->use_pairs && triples && ((r.flags & FFPAT_PLAN_THREE_STEP) || triples_preferred);
  }
  P->nvox = r.d.nvox();
  P->ndat = (size_t)r.n_angles * r.d.nz * r.ns;
  P->rows = r.n_angles * r.d.nz;
  P->lay = layout(r);

  e = hipMalloc(&P->base, P->lay.total);
  if (e != hipSuccess) {
    const size_t total = P->lay.total;
    delete P;
    (void)hipGetLastError();   // handled here: later launch checks must not see it
    return fail(FFPAT_ENOMEM, "hipMalloc(%zu) failed: %s", total, hipGetErrorString(e));
  }
  auto cleanup = [&](int code) {
    (void)hipStreamSynchronize(s);
    (void)hipFree(P->base);
    if (P->done) (void)hipEventDestroy(P->done);
    delete P;
    return code;
  };
  e = hipEventCreateWithFlags(&P->done, hipEventDisableTiming);
  if (e != hipSuccess) {
    P->done = nullptr;
    return cleanup(hip_fail(e, "hipEventCreateWithFlags"));
  }
  rc = apply_speed(P, c_dev, s);
  if (rc) return cleanup(rc);

  std::vector<AngleParams> ap((size_t)r.n_angles);
  std::vector<int> aorder;
  aorder.reserve((size_t)r.n_angles);
  for (int a = 0; a < r.n_angles; ++a) {
    ap[(size_t)a] = angle_params(geom->angles[a], r);
    if (ap[(size_t)a].hw > 1.0) P->two_tap = false;
    if (ap[(size_t)a].major_x) P->need_t = true;
    else {
      P->need_n = true;
      aorder.push_back(a);
    }
  }
  P->n_row_angles = (int)aorder.size();
  for (int a = 0; a < r.n_angles; ++a)
    if (ap[(size_t)a].major_x) aorder.push_back(a);
  // the pads of the padded copies stay zero for the life of the plan
  e = hipMemsetAsync(P->padN(), 0, P->lay.padN_bytes, s);
  if (e == hipSuccess) e = hipMemsetAsync(P->padT(), 0, P->lay.padT_bytes, s);
  if (e == hipSuccess) e = hipMemsetAsync(P->padD(), 0, P->lay.padD_bytes, s);
  if (e != hipSuccess) return cleanup(hip_fail(e, "plan memset"));
  if (is_f64(P)) {
    std::vector<double> t = ramp_taps<double>(r);
    e = hipMemcpyAsync(P->taps(), t.data(), t.size() * sizeof(double), hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipMemcpyAsync(P->ap(), ap.data(), ap.size() * sizeof(AngleParams), hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipMemcpyAsync(P->aorder(), aorder.data(), aorder.size() * sizeof(int), hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
  } else {
    std::vector<float> t = ramp_taps<float>(r);
    e = hipMemcpyAsync(P->taps(), t.data(), t.size() * sizeof(float), hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipMemcpyAsync(P->ap(), ap.data(), ap.size() * sizeof(AngleParams), hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipMemcpyAsync(P->aorder(), aorder.data(), aorder.size() * sizeof(int), hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
  }
  if (e != hipSuccess) return cleanup(hip_fail(e, "plan upload"));
  e = hipEventRecord(P->done, s);
  if (e != hipSuccess) return cleanup(hip_fail(e, "hipEventRecord"));
  *out = P;
  return FFPAT_OK;
}

int ffpat_plan_set_speed(ffpat_plan *plan, const void *c_dev, void *stream)
{
  TraceRange trace("ffpat_plan_set_speed");
  CHECK_PLAN(plan);
  CHECK_PTR(c_dev, "c_dev");
  DeviceGuard guard(plan->device);
  hipStream_t s = static_cast<hipStream_t>(stream);
  hipError_t e = hipEventSynchronize(plan->done);   // the plan's earlier work reads k'
  if (e != hipSuccess) return hip_fail(e, "hipEventSynchronize");
  const int nt_old = plan->nt;
  plan->has_step = false;            // the stored step belongs to the previous speed
  const int rc = apply_speed(plan, c_dev, s);
  if (rc) return rc;
  if (plan->nt != nt_old) {          // the captured launch sequences hold n_t steps
    if (plan->g_iter.exec) (void)hipGraphExecDestroy(plan->g_iter.exec);
    if (plan->g_power.exec) (void)hipGraphExecDestroy(plan->g_power.exec);
    plan->g_iter.exec = nullptr;
    plan->g_power.exec = nullptr;
  }
  return mark_done(plan, s, FFPAT_OK);
}

int ffpat_plan_info(const ffpat_plan *plan, int32_t *nt, double *dt, double *cmax)
{
  CHECK_PLAN(plan);
  if (nt) *nt = plan->nt;
  if (dt) *dt = plan->dt;
  if (cmax) *cmax = plan->cmax;
  return FFPAT_OK;
}

int ffpat_plan_steps_per_pass(const ffpat_plan *plan, int32_t *steps)
{
  CHECK_PLAN(plan);
  if (!steps) return fail(FFPAT_EINVAL, "steps is NULL");
  *steps = plan->use_triples ? 3 : (plan->use_pairs ? 2 : 1);
  return FFPAT_OK;
}

int ffpat_plan_stencil_shape(const ffpat_plan *plan, int32_t *tile_x, int32_t *tile_y, int32_t *zchunk)
{
  CHECK_PLAN(plan);
  int tx = 0, ty = 0, zc = 0;
  if (plan->stencil == STENCIL_BLOCKED) {
    DeviceGuard guard(plan->device);
    const size_t esz = plan->dtype == FFPAT_F64 ? 8 : 4;
    if (!plan->use_pairs) wave_step_shape(plan->d, esz, &tx, &ty, &zc);
    else if (plan->use_triples && esz == 8) wave_triple_shape<double>(plan->d, &tx, &ty, &zc);
    else if (plan->use_triples) wave_triple_shape<float>(plan->d, &tx, &ty, &zc);
    else if (esz == 8) wave_pair_shape<double>(plan->d, &tx, &ty, &zc);
    else wave_pair_shape<float>(plan->d, &tx, &ty, &zc);
  }
  if (tile_x) *tile_x = tx;
  if (tile_y) *tile_y = ty;
  if (zchunk) *zchunk = zc;
  return FFPAT_OK;
}

int ffpat_plan_destroy(ffpat_plan *plan)
{
  if (!plan) return FFPAT_OK;
  DeviceGuard guard(plan->device);
  const hipError_t e = hipEventSynchronize(plan->done);   // the plan's own work, not the device's
  if (plan->g_iter.exec) (void)hipGraphExecDestroy(plan->g_iter.exec);
  if (plan->g_power.exec) (void)hipGraphExecDestroy(plan->g_power.exec);
  if (plan->cap_stream) (void)hipStreamDestroy(plan->cap_stream);
  if (plan->obj) (void)hipFree(plan->obj);
  (void)hipFree(plan->base);
  (void)hipEventDestroy(plan->done);
  delete plan;
  if (e != hipSuccess) return hip_fail(e, "hipEventSynchronize");
  return FFPAT_OK;
}

#define DISPATCH(P, CALL_F, CALL_D) (is_f64(P) ? (CALL_D) : (CALL_F))

int ffpat_forward(ffpat_plan *plan, const void *h_dev, void *g_dev, void *stream)
{
  TraceRange trace("ffpat_forward");
  CHECK_PLAN(plan);
  CHECK_PTR(h_dev, "h_dev");
  CHECK_PTR(g_dev, "g_dev");
  DeviceGuard guard(plan->device);
  hipStream_t s = static_cast<hipStream_t>(stream);
  return mark_done(plan, s, DISPATCH(plan, op_forward<float>(plan, (const float *)h_dev, (float *)g_dev, s),
                                     op_forward<double>(plan, (const double *)h_dev, (double *)g_dev, s)));
}

int ffpat_adjoint(ffpat_plan *plan, const void *g_dev, void *h_dev, void *stream)
{
  TraceRange trace("ffpat_adjoint");
  CHECK_PLAN(plan);
  CHECK_PTR(h_dev, "h_dev");
  CHECK_PTR(g_dev, "g_dev");
  DeviceGuard guard(plan->device);
  hipStream_t s = static_cast<hipStream_t>(stream);
  return mark_done(plan, s, DISPATCH(plan, op_adjoint<float>(plan, (const float *)g_dev, (float *)h_dev, s),
                                     op_adjoint<double>(plan, (const double *)g_dev, (double *)h_dev, s)));
}

int ffpat_wave(ffpat_plan *plan, const void *h_dev, void *p_dev, void *stream)
{
  TraceRange trace("ffpat_wave");
  CHECK_PLAN(plan);
  CHECK_PTR(h_dev, "h_dev");
  CHECK_PTR(p_dev, "p_dev");
  if (h_dev == p_dev) return fail(FFPAT_EINVAL, "h_dev and p_dev must not overlap");
  DeviceGuard guard(plan->device);
  hipStream_t s = static_cast<hipStream_t>(stream);
  return mark_done(plan, s, DISPATCH(plan,
                  wave_forward<float>(plan, (const float *)h_dev, (float *)p_dev,
                                      Pool<float>{plan->vol(0), plan->vol(1), plan->vol(2), plan->vol(4)}, s),
                  wave_forward<double>(plan, (const double *)h_dev, (double *)p_dev,
                                       Pool<double>{plan->vol(0), plan->vol(1), plan->vol(2), plan->vol(4)}, s)));
}

int ffpat_wave_adjoint(ffpat_plan *plan, const void *g_dev, void *q_dev, void *stream)
{
  TraceRange trace("ffpat_wave_adjoint");
  CHECK_PLAN(plan);
  CHECK_PTR(g_dev, "g_dev");
  CHECK_PTR(q_dev, "q_dev");
  DeviceGuard guard(plan->device);
  hipStream_t s = static_cast<hipStream_t>(stream);
  return mark_done(plan, s, DISPATCH(plan, wave_adjoint_op<float>(plan, (const float *)g_dev, (float *)q_dev, s),
                                     wave_adjoint_op<double>(plan, (const double *)g_dev, (double *)q_dev, s)));
}

int ffpat_project(ffpat_plan *plan, const void *vol_dev, void *g_dev, void *stream)
{
  TraceRange trace("ffpat_project");
  CHECK_PLAN(plan);
  CHECK_PTR(vol_dev, "vol_dev");
  CHECK_PTR(g_dev, "g_dev");
  DeviceGuard guard(plan->device);
  hipStream_t s = static_cast<hipStream_t>(stream);
  hipError_t e = DISPATCH(plan, project<float>(plan, (const float *)vol_dev, (float *)g_dev, s),
                          project<double>(plan, (const double *)vol_dev, (double *)g_dev, s));
  return mark_done(plan, s, e == hipSuccess ? FFPAT_OK : hip_fail(e, "project"));
}

int ffpat_backproject(ffpat_plan *plan, const void *g_dev, void *vol_dev, void *stream)
{
  TraceRange trace("ffpat_backproject");
  CHECK_PLAN(plan);
  CHECK_PTR(vol_dev, "vol_dev");
  CHECK_PTR(g_dev, "g_dev");
  DeviceGuard guard(plan->device);
  hipStream_t s = static_cast<hipStream_t>(stream);
  hipError_t e = DISPATCH(plan, backproject_op<float>(plan, (const float *)g_dev, (float *)vol_dev, s),
                          backproject_op<double>(plan, (const double *)g_dev, (double *)vol_dev, s));
  return mark_done(plan, s, e == hipSuccess ? FFPAT_OK : hip_fail(e, "backproject"));
}

int ffpat_ramp(ffpat_plan *plan, const void *r_dev, void *y_dev, void *stream)
{
  TraceRange trace("ffpat_ramp");
  CHECK_PLAN(plan);
  CHECK_PTR(r_dev, "r_dev");
  CHECK_PTR(y_dev, "y_dev");
  DeviceGuard guard(plan->device);
  hipStream_t s = static_cast<hipStream_t>(stream);
  hipError_t e = DISPATCH(plan,
      launch_residual_ramp<float>(plan->rows, plan->ns, (const float *)r_dev, nullptr, nullptr, (const float *)plan->taps(), (float *)y_dev, plan->ns, 0, nullptr, s),
      launch_residual_ramp<double>(plan->rows, plan->ns, (const double *)r_dev, nullptr, nullptr, (const double *)plan->taps(), (double *)y_dev, plan->ns, 0, nullptr, s));
  return mark_done(plan, s, e == hipSuccess ? FFPAT_OK : hip_fail(e, "ramp"));
}

int ffpat_fbp(ffpat_plan *plan, const void *G_dev, void *vol_dev, void *stream)
{
  TraceRange trace("ffpat_fbp");
  CHECK_PLAN(plan);
  CHECK_PTR(G_dev, "G_dev");
  CHECK_PTR(vol_dev, "vol_dev");
  DeviceGuard guard(plan->device);
  hipStream_t s = static_cast<hipStream_t>(stream);
  return mark_done(plan, s, DISPATCH(plan, fbp_op<float>(plan, (const float *)G_dev, (float *)vol_dev, s),
                                     fbp_op<double>(plan, (const double *)G_dev, (double *)vol_dev, s)));
}

static int check_fb_args(ffpat_plan *plan, const void *G_dev, const ffpat_fb_params *params, void *h_dev)
{
  CHECK_PLAN(plan);
  CHECK_PTR(params, "params");
  CHECK_PTR(G_dev, "G_dev");
  CHECK_PTR(h_dev, "h_dev");
  if (params->n_iter < 0) return fail(FFPAT_EINVAL, "n_iter must be >= 0");
  if (params->n_power < 0) return fail(FFPAT_EINVAL, "n_power must be >= 0");
  if (!(params->lambda >= 0) || !std::isfinite(params->lambda)) return fail(FFPAT_EINVAL, "lambda must be finite and >= 0");
  if (!std::isfinite(params->step)) return fail(FFPAT_EINVAL, "step must be finite");
  if (params->cg_maxit < 0 || params->cg_maxit > 100000) return fail(FFPAT_EINVAL, "cg_maxit must be in [0, 100000]");
  if (!(params->cg_tol >= 0) || !std::isfinite(params->cg_tol)) return fail(FFPAT_EINVAL, "cg_tol must be >= 0");
  const uint32_t known = FFPAT_POSITIVITY | FFPAT_PRECOND | FFPAT_REG_GRAD | FFPAT_USE_PLAN_STEP | FFPAT_TWO_STEP;
  if (params->flags & ~known) return fail(FFPAT_EINVAL, "unknown flags 0x%x", (unsigned)(params->flags & ~known));
  if ((params->flags & FFPAT_TWO_STEP) && params->det_mask)
    return fail(FFPAT_EINVAL, "FFPAT_TWO_STEP works on volumes: det_mask must be NULL");
  if ((params->flags & FFPAT_REG_GRAD) && (params->flags & FFPAT_POSITIVITY))
    return fail(FFPAT_EINVAL, "FFPAT_REG_GRAD and FFPAT_POSITIVITY cannot be combined (no closed-form prox)");
  return FFPAT_OK;
}

int ffpat_reconstruct(ffpat_plan *plan, const void *G_dev, const ffpat_fb_params *params, void *h_dev,
                      double *step_used, void *stream)
{
  TraceRange trace("ffpat_reconstruct");
  int rc = check_fb_args(plan, G_dev, params, h_dev);
  if (rc) return rc;
  DeviceGuard guard(plan->device);
  hipStream_t s = static_cast<hipStream_t>(stream);
  return mark_done(plan, s, DISPATCH(plan,
                  reconstruct<float>(plan, (const float *)G_dev, params, (float *)h_dev, step_used, s),
                  reconstruct<double>(plan, (const double *)G_dev, params, (double *)h_dev, step_used, s)));
}

int ffpat_fb_enqueue(ffpat_plan *plan, const void *G_dev, const ffpat_fb_params *params, void *h_dev, void *stream)
{
  TraceRange trace("ffpat_fb_enqueue");
  int rc = check_fb_args(plan, G_dev, params, h_dev);
  if (rc) return rc;
  DeviceGuard guard(plan->device);
  hipStream_t s = static_cast<hipStream_t>(stream);
  return mark_done(plan, s, DISPATCH(plan, fb_enqueue<float>(plan, (const float *)G_dev, params, (float *)h_dev, s),
                                     fb_enqueue<double>(plan, (const double *)G_dev, params, (double *)h_dev, s)));
}

int ffpat_fb_enqueue_noalloc(ffpat_plan *plan, const void *G_dev, const ffpat_fb_params *params, void *h_dev,
                             void *stream)
{
  TraceRange trace("ffpat_fb_enqueue_noalloc");
  int rc = check_fb_args(plan, G_dev, params, h_dev);
  if (rc) return rc;
  if (params->n_iter > kNoAllocMaxIter)
    return fail(FFPAT_EINVAL, "n_iter %d exceeds the %d objective values the static history of "
                "ffpat_fb_enqueue_noalloc holds", params->n_iter, kNoAllocMaxIter);
  DeviceGuard guard(plan->device);
  double *history = scratch_address(plan->device);
  if (!history) {
    rc = scratch_resolve(plan->device);
    if (rc) return rc;
    history = scratch_address(plan->device);
  }
  hipStream_t s = static_cast<hipStream_t>(stream);
  return mark_done(plan, s,
                   DISPATCH(plan, fb_enqueue<float>(plan, (const float *)G_dev, params, (float *)h_dev, s, history),
                            fb_enqueue<double>(plan, (const double *)G_dev, params, (double *)h_dev, s, history)));
}

int ffpat_fb_report(ffpat_plan *plan, double *step_used, double *objective, int32_t n, void *stream)
{
  TraceRange trace("ffpat_fb_report");
  CHECK_PLAN(plan);
  if (n < 0) return fail(FFPAT_EINVAL, "n must be >= 0");
  if (n > 0 && !objective) return fail(FFPAT_EINVAL, "objective is NULL");
  DeviceGuard guard(plan->device);
  return fb_report(plan, step_used, objective, n, static_cast<hipStream_t>(stream));
}

}  // extern "C"
