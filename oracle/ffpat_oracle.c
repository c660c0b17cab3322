/*
 * FP64 CPU oracle for one-step full-field photoacoustic reconstruction
 * (Haltmeier, Zangerl, Nuster, Nguyen, "Photoacoustic image reconstruction
 * from full field data in heterogeneous media", 2019).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the plain, slow, obviously correct
 * definition that the HIP library is checked against.  Only the test suite,
 * the smoke check and the CPU-baseline leg of the benchmark may load it.  It
 * shares no code, header, table or constant with the HIP path.
 *
 * Everything is double precision, written as direct loops over the
 * definitions; OpenMP only splits independent outer loops.
 *
 * Discrete model (readings of the paper are listed in the design notes):
 *   grid      node-centred, x_i = (i - (nx-1)/2) dx, same for y, z; arrays
 *             [nz][ny][nx], x fastest.  The rotation axis is the grid's
 *             z axis through its centre.
 *   W_T       wave equation (Sec. 2.1, eq. wave1/wave2): leapfrog in time,
 *             fourth-order 13-point Laplacian with zero values outside the
 *             grid, zero initial velocity via the symmetric first step
 *             p1 = p0 + (1/2) kappa L p0, kappa = (c dt)^2.
 *   X         X-ray transform in each plane z = const (eq. Radon), with
 *             linear interpolation along the minor axis (Sec. 4.1), written
 *             as a per-voxel triangular footprint on the detector.
 *   Lambda    ramp filter |omega| along the detector coordinate (Sec. 3.1),
 *             as the discrete Ram-Lak Toeplitz kernel, scaled so that
 *             X^T Lambda X approximates the identity (filtered
 *             backprojection, Sec. 3.1).
 *   FB        Algorithm 8 (Sec. 3.2) with prox of
 *             R = 1/2 ||h||^2 + indicator(h >= 0), or R = 1/2 ||grad h||^2.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifndef M_PI
#define M_PI 3.14159265358979323846
#endif

typedef struct {
  int32_t nx, ny, nz;
  int32_t ndim;          /* 3: Laplacian over x,y,z; 2: over x,y only (z-invariant mode, Sec. 4) */
  double dx;             /* isotropic grid spacing */
  double T;              /* final measurement time */
  double cfl;            /* c_max dt / dx target */
  int32_t n_angles;
  const double *angles;  /* radians */
  int32_t ns;            /* detector bins per row */
  double ds;             /* detector spacing */
} orc_geom;

enum {
  ORC_POSITIVITY = 1u,   /* R includes the indicator of h >= 0 */
  ORC_PRECOND = 2u,      /* use Lambda in the data term (else identity) */
  ORC_REG_GRAD = 4u      /* R = 1/2 ||D h||^2 instead of 1/2 ||h||^2 */
};

static size_t nvox(const orc_geom *g) { return (size_t)g->nx * g->ny * g->nz; }
static size_t ndat(const orc_geom *g) { return (size_t)g->n_angles * g->nz * g->ns; }

/* ------------------------------------------------------------------------ */
/* Time grid: dt = cfl dx / c_max rounded so that n_t dt = T exactly.         */
/* ------------------------------------------------------------------------ */
int orc_time_grid(double T, double cmax, double cfl, double dx, int32_t *nt, double *dt)
{
  double x = T * cmax / (cfl * dx);
  double n = ceil(x * (1.0 - 1e-12));
  if (n < 1.0) n = 1.0;
  *nt = (int32_t)n;
  *dt = T / n;
  return 0;
}

double orc_max(const double *a, size_t n)
{
  double m = -INFINITY;
  for (size_t i = 0; i < n; ++i)
    if (a[i] > m) m = a[i];
  return m;
}

/* ------------------------------------------------------------------------ */
/* Fourth-order Laplacian, zero outside the grid.                             */
/* (L f)_p = sum over axes of (-f[-2] + 16 f[-1] - 30 f[0] + 16 f[+1] - f[+2]) */
/*           / (12 dx^2)                                                       */
/* ------------------------------------------------------------------------ */
static double at(const orc_geom *g, const double *f, long z, long y, long x)
{
  if (x < 0 || y < 0 || z < 0 || x >= g->nx || y >= g->ny || z >= g->nz) return 0.0;
  return f[((size_t)z * g->ny + (size_t)y) * g->nx + (size_t)x];
}

static const double stencil4[5] = {-1.0, 16.0, -30.0, 16.0, -1.0};

void orc_laplacian(const orc_geom *g, const double *f, double *out)
{
  const double inv = 1.0 / (12.0 * g->dx * g->dx);
  #pragma omp parallel for collapse(2) schedule(static)
  for (long z = 0; z < g->nz; ++z)
    for (long y = 0; y < g->ny; ++y)
      for (long x = 0; x < g->nx; ++x) {
        double acc = 0.0;
        for (int o = -2; o <= 2; ++o) {
          acc += stencil4[o + 2] * at(g, f, z, y, x + o);
          acc += stencil4[o + 2] * at(g, f, z, y + o, x);
          if (g->ndim == 3) acc += stencil4[o + 2] * at(g, f, z + o, y, x);
        }
        out[((size_t)z * g->ny + y) * g->nx + x] = acc * inv;
      }
}

/* kappa = (c dt)^2 with dt from the time grid */
static int make_kappa(const orc_geom *g, const double *c, double *kappa, int32_t *nt_out, double *dt_out)
{
  size_t n = nvox(g);
  int32_t nt; double dt;
  orc_time_grid(g->T, orc_max(c, n), g->cfl, g->dx, &nt, &dt);
  for (size_t i = 0; i < n; ++i) kappa[i] = (c[i] * dt) * (c[i] * dt);
  if (nt_out) *nt_out = nt;
  if (dt_out) *dt_out = dt;
  return nt;
}

int orc_plan_info(const orc_geom *g, const double *c, int32_t *nt, double *dt, double *cmax)
{
  *cmax = orc_max(c, nvox(g));
  return orc_time_grid(g->T, *cmax, g->cfl, g->dx, nt, dt);
}

/* ------------------------------------------------------------------------ */
/* W_T h = p(., T): p0 = h, dp/dt(0) = 0 (eq. wave2).                          */
/*   p1      = p0 + 1/2 kappa L p0                                              */
/*   p(k+1)  = 2 p(k) - p(k-1) + kappa L p(k)                                   */
/* ------------------------------------------------------------------------ */
int orc_wave(const orc_geom *g, const double *c, const double *h, double *out)
{
  size_t n = nvox(g);
  double *kappa = malloc(n * sizeof(double));
  double *prev = malloc(n * sizeof(double));
  double *cur = malloc(n * sizeof(double));
  double *lap = malloc(n * sizeof(double));
  if (!kappa || !prev || !cur || !lap) { free(kappa); free(prev); free(cur); free(lap); return -3; }
  int32_t nt = make_kappa(g, c, kappa, NULL, NULL);

  memcpy(prev, h, n * sizeof(double));
  orc_laplacian(g, prev, lap);
  for (size_t i = 0; i < n; ++i) cur[i] = prev[i] + 0.5 * kappa[i] * lap[i];
  for (int32_t k = 1; k < nt; ++k) {
    orc_laplacian(g, cur, lap);
    #pragma omp parallel for schedule(static)
    for (size_t i = 0; i < n; ++i) {
      double next = 2.0 * cur[i] - prev[i] + kappa[i] * lap[i];
      prev[i] = cur[i];
      cur[i] = next;
    }
  }
  memcpy(out, cur, n * sizeof(double));
  free(kappa); free(prev); free(cur); free(lap);
  return 0;
}

/* ------------------------------------------------------------------------ */
/* Euclidean transpose of W_T (Sec. 3.1, adjoint wave operator).  The scheme  */
/* is p(n) = P_n(K L) h with K = diag(kappa); its transpose is P_n(L K),     */
/* i.e. the same recursion with kappa applied before the Laplacian:           */
/*   q1      = q0 + 1/2 L(kappa q0)                                             */
/*   q(k+1)  = 2 q(k) - q(k-1) + L(kappa q(k))                                  */
/* ------------------------------------------------------------------------ */
int orc_wave_T(const orc_geom *g, const double *c, const double *gin, double *out)
{
  size_t n = nvox(g);
  double *kappa = malloc(n * sizeof(double));
  double *prev = malloc(n * sizeof(double));
  double *cur = malloc(n * sizeof(double));
  double *tmp = malloc(n * sizeof(double));
  double *lap = malloc(n * sizeof(double));
  if (!kappa || !prev || !cur || !tmp || !lap) {
    free(kappa); free(prev); free(cur); free(tmp); free(lap); return -3;
  }
  int32_t nt = make_kappa(g, c, kappa, NULL, NULL);

  memcpy(prev, gin, n * sizeof(double));
  for (size_t i = 0; i < n; ++i) tmp[i] = kappa[i] * prev[i];
  orc_laplacian(g, tmp, lap);
  for (size_t i = 0; i < n; ++i) cur[i] = prev[i] + 0.5 * lap[i];
  for (int32_t k = 1; k < nt; ++k) {
    for (size_t i = 0; i < n; ++i) tmp[i] = kappa[i] * cur[i];
    orc_laplacian(g, tmp, lap);
    #pragma omp parallel for schedule(static)
    for (size_t i = 0; i < n; ++i) {
      double next = 2.0 * cur[i] - prev[i] + lap[i];
      prev[i] = cur[i];
      cur[i] = next;
    }
  }
  memcpy(out, cur, n * sizeof(double));
  free(kappa); free(prev); free(cur); free(tmp); free(lap);
  return 0;
}

/* ------------------------------------------------------------------------ */
/* X-ray transform per plane z (eq. Radon):                                   */
/*   (X phi)(theta, s, z) = integral of phi(s theta + t theta_perp, z) dt,      */
/* theta = (cos a, sin a).  Discretised with linear interpolation along the   */
/* minor axis: a voxel at (x, y) with t = x cos a + y sin a reaches detector  */
/* bin s_j with weight (dx/m) max(0, 1 - |s_j - t| / (m dx)),                 */
/* m = max(|cos a|, |sin a|).                                                 */
/* ------------------------------------------------------------------------ */
static double coord(long i, int32_t n, double h) { return ((double)i - 0.5 * (n - 1)) * h; }

/* Detector bins that can lie within `half` of position t (one spare bin on
 * each side; the weight test itself decides), clipped to the detector. */
static void bin_range(const orc_geom *g, double t, double half, long *lo, long *hi)
{
  const double c0 = 0.5 * (g->ns - 1);
  long a = (long)floor((t - half) / g->ds + c0) - 1;
  long b = (long)ceil((t + half) / g->ds + c0) + 1;
  *lo = a < 0 ? 0 : a;
  *hi = b > g->ns - 1 ? g->ns - 1 : b;
}

void orc_project(const orc_geom *g, const double *vol, double *data)
{
  memset(data, 0, ndat(g) * sizeof(double));
  #pragma omp parallel for schedule(dynamic)
  for (long a = 0; a < g->n_angles; ++a) {
    const double ca = cos(g->angles[a]), sa = sin(g->angles[a]);
    const double m = fmax(fabs(ca), fabs(sa));
    const double half = m * g->dx;           /* footprint half-width */
    for (long z = 0; z < g->nz; ++z) {
      double *row = data + ((size_t)a * g->nz + z) * g->ns;
      for (long k = 0; k < g->ny; ++k)
        for (long i = 0; i < g->nx; ++i) {
          const double v = vol[((size_t)z * g->ny + k) * g->nx + i];
          const double t = coord(i, g->nx, g->dx) * ca + coord(k, g->ny, g->dx) * sa;
          long jlo, jhi;
          bin_range(g, t, half, &jlo, &jhi);
          for (long j = jlo; j <= jhi; ++j) {
            const double d = fabs(coord(j, g->ns, g->ds) - t);
            if (d < half) row[j] += (g->dx / m) * (1.0 - d / half) * v;
          }
        }
    }
  }
}

/* Transpose of orc_project: the same weights gathered per voxel. */
void orc_backproject(const orc_geom *g, const double *data, double *vol)
{
  double *cs = malloc(2 * (size_t)g->n_angles * sizeof(double));
  if (!cs) return;
  for (long a = 0; a < g->n_angles; ++a) { cs[2 * a] = cos(g->angles[a]); cs[2 * a + 1] = sin(g->angles[a]); }
  #pragma omp parallel for collapse(2) schedule(static)
  for (long z = 0; z < g->nz; ++z)
    for (long k = 0; k < g->ny; ++k)
      for (long i = 0; i < g->nx; ++i) {
        double acc = 0.0;
        for (long a = 0; a < g->n_angles; ++a) {
          const double ca = cs[2 * a], sa = cs[2 * a + 1];
          const double m = fmax(fabs(ca), fabs(sa));
          const double half = m * g->dx;
          const double t = coord(i, g->nx, g->dx) * ca + coord(k, g->ny, g->dx) * sa;
          const double *row = data + ((size_t)a * g->nz + z) * g->ns;
          long jlo, jhi;
          bin_range(g, t, half, &jlo, &jhi);
          for (long j = jlo; j <= jhi; ++j) {
            const double d = fabs(coord(j, g->ns, g->ds) - t);
            if (d < half) acc += (g->dx / m) * (1.0 - d / half) * row[j];
          }
        }
        vol[((size_t)z * g->ny + k) * g->nx + i] = acc;
      }
  free(cs);
}

/* ------------------------------------------------------------------------ */
/* Preconditioner Lambda (Sec. 3.1): ramp filter along the detector coordinate.*/
/* Ram-Lak samples h0 = 1/4, h_n = -1/(pi n)^2 for odd n, 0 for even n != 0,   */
/* finite Toeplitz section per detector row, times pi / (N_angles dx^2).       */
/* ------------------------------------------------------------------------ */
double orc_ramlak_tap(long n)
{
  if (n == 0) return 0.25;
  if (n % 2 == 0) return 0.0;
  return -1.0 / (M_PI * M_PI * (double)n * (double)n);
}

double orc_ramp_scale(const orc_geom *g) { return M_PI / ((double)g->n_angles * g->dx * g->dx); }

void orc_ramp(const orc_geom *g, const double *r, double *y)
{
  const double C = orc_ramp_scale(g);
  const long rows = (long)g->n_angles * g->nz;
  #pragma omp parallel for schedule(static)
  for (long row = 0; row < rows; ++row) {
    const double *rr = r + (size_t)row * g->ns;
    double *yy = y + (size_t)row * g->ns;
    for (long j = 0; j < g->ns; ++j) {
      double acc = 0.0;
      for (long jj = 0; jj < g->ns; ++jj) acc += orc_ramlak_tap(j - jj) * rr[jj];
      yy[j] = C * acc;
    }
  }
}

/* A = X W_T and its transpose A^T = W_T^T X^T. */
int orc_forward(const orc_geom *g, const double *c, const double *h, double *data)
{
  double *p = malloc(nvox(g) * sizeof(double));
  if (!p) return -3;
  int rc = orc_wave(g, c, h, p);
  if (rc == 0) orc_project(g, p, data);
  free(p);
  return rc;
}

int orc_adjoint(const orc_geom *g, const double *c, const double *data, double *h)
{
  double *b = malloc(nvox(g) * sizeof(double));
  if (!b) return -3;
  orc_backproject(g, data, b);
  int rc = orc_wave_T(g, c, b, h);
  free(b);
  return rc;
}

/* ------------------------------------------------------------------------ */
/* Gradient regulariser R(h) = 1/2 ||D h||^2, D = forward differences / dx    */
/* with zero values outside the grid; D^T D = -(7-point Laplacian).          */
/* prox_{tau R}(f) solves (I + tau D^T D) h = f; plain conjugate gradients.  */
/* ------------------------------------------------------------------------ */
void orc_neg_lap7(const orc_geom *g, const double *f, double *out)
{
  const double inv = 1.0 / (g->dx * g->dx);
  #pragma omp parallel for collapse(2) schedule(static)
  for (long z = 0; z < g->nz; ++z)
    for (long y = 0; y < g->ny; ++y)
      for (long x = 0; x < g->nx; ++x) {
        double acc = 2.0 * at(g, f, z, y, x) - at(g, f, z, y, x - 1) - at(g, f, z, y, x + 1);
        acc += 2.0 * at(g, f, z, y, x) - at(g, f, z, y - 1, x) - at(g, f, z, y + 1, x);
        if (g->ndim == 3) acc += 2.0 * at(g, f, z, y, x) - at(g, f, z - 1, y, x) - at(g, f, z + 1, y, x);
        out[((size_t)z * g->ny + y) * g->nx + x] = acc * inv;
      }
}

double orc_dot(const double *a, const double *b, size_t n)
{
  double s = 0.0;
  for (size_t i = 0; i < n; ++i) s += a[i] * b[i];
  return s;
}

/* Solves (I + tau D^T D) h = f by CG from h = f, until ||res|| <= tol ||f|| or maxit. */
int orc_prox_grad(const orc_geom *g, double tau, const double *f, double *h, double tol, int32_t maxit)
{
  size_t n = nvox(g);
  double *r = malloc(n * sizeof(double)), *p = malloc(n * sizeof(double)), *Ap = malloc(n * sizeof(double));
  if (!r || !p || !Ap) { free(r); free(p); free(Ap); return -3; }
  memcpy(h, f, n * sizeof(double));
  orc_neg_lap7(g, h, Ap);
  for (size_t i = 0; i < n; ++i) { r[i] = f[i] - (h[i] + tau * Ap[i]); p[i] = r[i]; }
  double rr = orc_dot(r, r, n);
  const double stop = tol * tol * orc_dot(f, f, n);
  int32_t it = 0;
  while (rr > stop && it < maxit) {
    orc_neg_lap7(g, p, Ap);
    for (size_t i = 0; i < n; ++i) Ap[i] = p[i] + tau * Ap[i];
    const double alpha = rr / orc_dot(p, Ap, n);
    for (size_t i = 0; i < n; ++i) { h[i] += alpha * p[i]; r[i] -= alpha * Ap[i]; }
    const double rr_new = orc_dot(r, r, n);
    for (size_t i = 0; i < n; ++i) p[i] = r[i] + (rr_new / rr) * p[i];
    rr = rr_new;
    ++it;
  }
  free(r); free(p); free(Ap);
  return it;
}

/* ------------------------------------------------------------------------ */
/* Data-term pieces shared by the power iteration and FB:                     */
/*   r = chi_M (A h - G),  y = chi_M Lambda r  (Lambda = I without PRECOND)    */
/* ------------------------------------------------------------------------ */
static void apply_mask(const uint8_t *mask, double *d, size_t n)
{
  if (!mask) return;
  for (size_t i = 0; i < n; ++i)
    if (!mask[i]) d[i] = 0.0;
}

/* w = A^T chi_M Lambda chi_M A v  (the Hessian of the data term) */
static int normal_op(const orc_geom *g, const double *c, uint32_t flags, const uint8_t *det_mask,
                     const double *v, double *w, double *dat, double *dat2)
{
  size_t nd = ndat(g);
  int rc = orc_forward(g, c, v, dat);
  if (rc) return rc;
  apply_mask(det_mask, dat, nd);
  if (flags & ORC_PRECOND) orc_ramp(g, dat, dat2);
  else memcpy(dat2, dat, nd * sizeof(double));
  apply_mask(det_mask, dat2, nd);
  return orc_adjoint(g, c, dat2, w);
}

/* Power iteration: v0 = ones/||ones||, w = H v, L = ||w||, v = w / L.
 * Returns L after n_power steps in *L_out (step size 1/L). */
int orc_power(const orc_geom *g, const double *c, uint32_t flags, const uint8_t *det_mask,
              int32_t n_power, double *L_out, double *L_hist)
{
  size_t n = nvox(g), nd = ndat(g);
  double *v = malloc(n * sizeof(double)), *w = malloc(n * sizeof(double));
  double *d1 = malloc(nd * sizeof(double)), *d2 = malloc(nd * sizeof(double));
  if (!v || !w || !d1 || !d2) { free(v); free(w); free(d1); free(d2); return -3; }
  for (size_t i = 0; i < n; ++i) v[i] = 1.0 / sqrt((double)n);
  double L = 0.0;
  int rc = 0;
  for (int32_t it = 0; it < n_power; ++it) {
    rc = normal_op(g, c, flags, det_mask, v, w, d1, d2);
    if (rc) break;
    L = sqrt(orc_dot(w, w, n));
    if (L_hist) L_hist[it] = L;
    for (size_t i = 0; i < n; ++i) v[i] = w[i] / L;
  }
  *L_out = L;
  free(v); free(w); free(d1); free(d2);
  return rc;
}

/* ------------------------------------------------------------------------ */
/* Algorithm 8: preconditioned proximal forward-backward splitting.          */
/*   r_k     = chi_M (A h_k - G)                                               */
/*   J_k     = 1/2 <Lambda r_k, r_k> + lambda R(h_k)   (evaluated at h_k)      */
/*   f       = h_k - s A^T chi_M Lambda r_k                                    */
/*   h_{k+1} = prox_{s lambda R}(f)                                            */
/* h holds h_0 on entry (zeros reproduce the paper's start) and h_K on exit. */
/* step <= 0 selects s = 1 / L from n_power power-iteration steps.           */
/* ------------------------------------------------------------------------ */
int orc_fb(const orc_geom *g, const double *c, const double *G, double lambda, double step,
           int32_t n_iter, int32_t n_power, uint32_t flags, const uint8_t *support,
           const uint8_t *det_mask, double *h, double *objective, double *step_used)
{
  size_t n = nvox(g), nd = ndat(g);
  int rc = 0;
  double s = step;
  if (s <= 0.0) {
    double L;
    rc = orc_power(g, c, flags, det_mask, n_power > 0 ? n_power : 20, &L, NULL);
    if (rc) return rc;
    s = 1.0 / L;
  }
  if (step_used) *step_used = s;

  double *r = malloc(nd * sizeof(double)), *y = malloc(nd * sizeof(double));
  double *grad = malloc(n * sizeof(double)), *f = malloc(n * sizeof(double));
  double *tmp = malloc(n * sizeof(double));
  if (!r || !y || !grad || !f || !tmp) { free(r); free(y); free(grad); free(f); free(tmp); return -3; }

  for (int32_t k = 0; k < n_iter && rc == 0; ++k) {
    rc = orc_forward(g, c, h, r);
    if (rc) break;
    for (size_t i = 0; i < nd; ++i) r[i] -= G[i];
    apply_mask(det_mask, r, nd);
    if (flags & ORC_PRECOND) orc_ramp(g, r, y);
    else memcpy(y, r, nd * sizeof(double));
    apply_mask(det_mask, y, nd);

    if (objective) {
      double reg;
      if (flags & ORC_REG_GRAD) {
        orc_neg_lap7(g, h, tmp);
        reg = 0.5 * orc_dot(h, tmp, n);
      } else {
        reg = 0.5 * orc_dot(h, h, n);
      }
      objective[k] = 0.5 * orc_dot(r, y, nd) + lambda * reg;
    }

    rc = orc_adjoint(g, c, y, grad);
    if (rc) break;
    for (size_t i = 0; i < n; ++i) f[i] = h[i] - s * grad[i];

    if (flags & ORC_REG_GRAD) {
      int it = orc_prox_grad(g, s * lambda, f, h, 1e-13, 10000);
      if (it < 0) { rc = it; break; }
      if (support) for (size_t i = 0; i < n; ++i) if (!support[i]) h[i] = 0.0;
    } else {
      for (size_t i = 0; i < n; ++i) {
        double v = f[i];
        if ((flags & ORC_POSITIVITY) && v < 0.0) v = 0.0;
        v = v / (1.0 + s * lambda);
        if (support && !support[i]) v = 0.0;
        h[i] = v;
      }
    }
  }
  free(r); free(y); free(grad); free(f); free(tmp);
  return rc;
}

/* Discrete energy of the leapfrog scheme between levels k and k+1:
 *   E = sum (p1 - p0)^2 / kappa - p1^T L p0,
 * conserved exactly (in exact arithmetic) by the recursion above. */
double orc_energy(const orc_geom *g, const double *c, const double *p0, const double *p1)
{
  size_t n = nvox(g);
  double *kappa = malloc(n * sizeof(double)), *lap = malloc(n * sizeof(double));
  if (!kappa || !lap) { free(kappa); free(lap); return NAN; }
  make_kappa(g, c, kappa, NULL, NULL);
  orc_laplacian(g, p0, lap);
  double e = 0.0;
  for (size_t i = 0; i < n; ++i) e += (p1[i] - p0[i]) * (p1[i] - p0[i]) / kappa[i] - p1[i] * lap[i];
  free(kappa); free(lap);
  return e;
}

/* Wave states p(k) for k = 0..nsteps (for energy and time-reversal tests). */
int orc_wave_history(const orc_geom *g, const double *c, const double *h, int32_t nsteps, double *hist)
{
  size_t n = nvox(g);
  double *kappa = malloc(n * sizeof(double)), *lap = malloc(n * sizeof(double));
  if (!kappa || !lap) { free(kappa); free(lap); return -3; }
  make_kappa(g, c, kappa, NULL, NULL);
  memcpy(hist, h, n * sizeof(double));
  if (nsteps >= 1) {
    orc_laplacian(g, hist, lap);
    for (size_t i = 0; i < n; ++i) hist[n + i] = hist[i] + 0.5 * kappa[i] * lap[i];
  }
  for (int32_t k = 1; k < nsteps; ++k) {
    const double *cur = hist + (size_t)k * n, *prev = hist + (size_t)(k - 1) * n;
    double *next = hist + (size_t)(k + 1) * n;
    orc_laplacian(g, cur, lap);
    for (size_t i = 0; i < n; ++i) next[i] = 2.0 * cur[i] - prev[i] + kappa[i] * lap[i];
  }
  free(kappa); free(lap);
  return 0;
}

/* ------------------------------------------------------------------------ */
/* Filtered backprojection X^-1 = X^* Lambda (Sec. 3.1), plane by plane.     */
/* ------------------------------------------------------------------------ */
int orc_fbp(const orc_geom *g, const double *G, double *vol)
{
  double *y = malloc(ndat(g) * sizeof(double));
  if (!y) return -3;
  orc_ramp(g, G, y);
  orc_backproject(g, y, vol);
  free(y);
  return 0;
}

/* ------------------------------------------------------------------------ */
/* Algorithm 9 (Sec. 4.1): the second stage of the two-step method,         */
/* forward-backward splitting on 1/2 ||W_T h - g||^2 + lambda R(h) with g a  */
/* volume (the first stage is g = X^-1 G).  Same prox and step rules as      */
/* orc_fb; the power iteration runs on W_T^T W_T.                           */
/* ------------------------------------------------------------------------ */
int orc_fb_two_step(const orc_geom *g, const double *c, const double *gvol, double lambda, double step,
                    int32_t n_iter, int32_t n_power, uint32_t flags, const uint8_t *support, double *h,
                    double *objective, double *step_used)
{
  size_t n = nvox(g);
  int rc = 0;
  double *r = malloc(n * sizeof(double)), *grad = malloc(n * sizeof(double));
  double *f = malloc(n * sizeof(double)), *tmp = malloc(n * sizeof(double));
  if (!r || !grad || !f || !tmp) { free(r); free(grad); free(f); free(tmp); return -3; }
  double s = step;
  if (s <= 0.0) {
    /* power iteration on W^T W from the normalised all-ones vector */
    for (size_t i = 0; i < n; ++i) f[i] = 1.0 / sqrt((double)n);
    double L = 0.0;
    for (int32_t it = 0; it < (n_power > 0 ? n_power : 20); ++it) {
      rc = orc_wave(g, c, f, r);
      if (!rc) rc = orc_wave_T(g, c, r, grad);
      if (rc) break;
      L = sqrt(orc_dot(grad, grad, n));
      for (size_t i = 0; i < n; ++i) f[i] = grad[i] / L;
    }
    s = 1.0 / L;
  }
  if (step_used) *step_used = s;
  for (int32_t k = 0; k < n_iter && rc == 0; ++k) {
    rc = orc_wave(g, c, h, r);
    if (rc) break;
    for (size_t i = 0; i < n; ++i) r[i] -= gvol[i];
    if (objective) {
      double reg;
      if (flags & ORC_REG_GRAD) {
        orc_neg_lap7(g, h, tmp);
        reg = 0.5 * orc_dot(h, tmp, n);
      } else {
        reg = 0.5 * orc_dot(h, h, n);
      }
      objective[k] = 0.5 * orc_dot(r, r, n) + lambda * reg;
    }
    rc = orc_wave_T(g, c, r, grad);
    if (rc) break;
    for (size_t i = 0; i < n; ++i) f[i] = h[i] - s * grad[i];
    if (flags & ORC_REG_GRAD) {
      int it = orc_prox_grad(g, s * lambda, f, h, 1e-13, 10000);
      if (it < 0) { rc = it; break; }
      if (support) for (size_t i = 0; i < n; ++i) if (!support[i]) h[i] = 0.0;
    } else {
      for (size_t i = 0; i < n; ++i) {
        double v = f[i];
        if ((flags & ORC_POSITIVITY) && v < 0.0) v = 0.0;
        v = v / (1.0 + s * lambda);
        if (support && !support[i]) v = 0.0;
        h[i] = v;
      }
    }
  }
  free(r); free(grad); free(f); free(tmp);
  return rc;
}
