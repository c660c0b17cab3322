// Forward-backward (Algorithm 8, Sec. 3.2) element-wise updates and the FP64
// reductions behind the objective, the norms and the power iteration.
//
// Reductions are deterministic: a fixed grid of kReduceBlocks work-groups
// writes one FP64 partial each (fixed-order tree inside the group), and a
// single work-group adds the partials in a fixed order.  No atomics, so a
// result does not depend on scheduling or on other work sharing the GPU.
#include "kernels.h"

namespace ffpat {

__device__ inline double block_sum_256(double v, double *red)
{
  red[threadIdx.x] = v;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  return red[0];
}

template <typename T>
__global__ void __launch_bounds__(256) sumsq_kernel(const T *__restrict__ x, size_t n, double *partials)
{
  __shared__ double red[256];
  double acc = 0.0;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
    const double v = (double)x[i];
    acc += v * v;
  }
  const double t = block_sum_256(acc, red);
  if (threadIdx.x == 0) partials[blockIdx.x] = t;
}

template <typename T>
__global__ void __launch_bounds__(256)
dot_kernel(const T *__restrict__ x, const T *__restrict__ y, size_t n, double *partials)
{
  __shared__ double red[256];
  double acc = 0.0;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    acc += (double)x[i] * (double)y[i];
  const double t = block_sum_256(acc, red);
  if (threadIdx.x == 0) partials[blockIdx.x] = t;
}

template <typename T>
hipError_t launch_sumsq(const T *x, size_t n, double *partials, hipStream_t s)
{
  sumsq_kernel<T><<<kReduceBlocks, kReduceThreads, 0, s>>>(x, n, partials);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_dot(const T *x, const T *y, size_t n, double *partials, hipStream_t s)
{
  dot_kernel<T><<<kReduceBlocks, kReduceThreads, 0, s>>>(x, y, n, partials);
  return hipGetLastError();
}

__global__ void __launch_bounds__(256) reduce_to_kernel(const double *partials, int n, double scale, double *out)
{
  __shared__ double red[256];
  double acc = 0.0;
  for (int i = threadIdx.x; i < n; i += blockDim.x) acc += partials[i];
  const double t = block_sum_256(acc, red);
  if (threadIdx.x == 0) out[0] = scale * t;
}

hipError_t launch_reduce_to(const double *partials, int n, double scale, double *out, hipStream_t s)
{
  reduce_to_kernel<<<1, 256, 0, s>>>(partials, n, scale, out);
  return hipGetLastError();
}

__global__ void objective_kernel(const double *data_sum, const double *reg_sum, double lambda, double *obj,
                                 double *counter, int capacity, double *nonfinite)
{
  if (threadIdx.x == 0) {
    const double d = data_sum[0];
    const double r = reg_sum[0];
    const double J = 0.5 * d + lambda * 0.5 * r;
    const int k = (int)counter[0];
    if (k < capacity) obj[k] = J;
    counter[0] = (double)(k + 1);
    if (!isfinite(J)) nonfinite[0] = 1.0;
  }
}

hipError_t launch_objective(const double *data_sum, const double *reg_sum, double lambda, double *obj,
                            double *counter, int capacity, double *nonfinite, hipStream_t s)
{
  objective_kernel<<<1, 64, 0, s>>>(data_sum, reg_sum, lambda, obj, counter, capacity, nonfinite);
  return hipGetLastError();
}

__global__ void power_finish_kernel(const double *sumsq, double *L, double *step, double *nonfinite)
{
  if (threadIdx.x == 0) {
    const double l = sqrt(sumsq[0]);
    L[0] = l;
    step[0] = 1.0 / l;
    if (!isfinite(l) || !(l > 0.0)) nonfinite[0] = 1.0;
  }
}

hipError_t launch_power_finish(const double *sumsq, double *L, double *step, double *nonfinite, hipStream_t s)
{
  power_finish_kernel<<<1, 64, 0, s>>>(sumsq, L, step, nonfinite);
  return hipGetLastError();
}

template <typename T>
__global__ void fill_kernel(T *x, size_t n, T v)
{
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) x[i] = v;
}

template <typename T>
hipError_t launch_fill(T *x, size_t n, double value, hipStream_t s)
{
  fill_kernel<T><<<1024, 256, 0, s>>>(x, n, (T)value);
  return hipGetLastError();
}

template <typename T>
__global__ void normalize_kernel(const T *x, T *y, size_t n, const double *sumsq)
{
  const T inv = (T)(1.0 / sqrt(sumsq[0]));
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    y[i] = x[i] * inv;
}

template <typename T>
hipError_t launch_normalize(const T *x, T *y, size_t n, const double *sumsq, hipStream_t s)
{
  normalize_kernel<T><<<1024, 256, 0, s>>>(x, y, n, sumsq);
  return hipGetLastError();
}

// prox of s lambda (1/2 ||h||^2 + indicator(h >= 0)): h = max(f, 0) / (1 + s lambda)
template <typename T>
__global__ void prox_l2_kernel(T *h, const T *__restrict__ grad, size_t n, const double *step, double lambda,
                               int positivity, const uint8_t *__restrict__ support)
{
  const double s = step[0];
  const T sT = (T)s;
  const T inv = (T)(1.0 / (1.0 + s * lambda));
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
    T f = h[i] - sT * grad[i];
    if (positivity && f < T(0)) f = T(0);
    f = f * inv;
    if (support && !support[i]) f = T(0);
    h[i] = f;
  }
}

template <typename T>
hipError_t launch_prox_l2(T *h, const T *grad, size_t n, const double *step, double lambda, int positivity,
                          const uint8_t *support, hipStream_t s)
{
  prox_l2_kernel<T><<<2048, 256, 0, s>>>(h, grad, n, step, lambda, positivity, support);
  return hipGetLastError();
}

template <typename T>
__global__ void grad_step_kernel(const T *h, const T *__restrict__ grad, T *f, size_t n, const double *step)
{
  const T sT = (T)step[0];
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    f[i] = h[i] - sT * grad[i];
}

template <typename T>
hipError_t launch_grad_step(const T *h, const T *grad, T *f, size_t n, const double *step, hipStream_t s)
{
  grad_step_kernel<T><<<2048, 256, 0, s>>>(h, grad, f, n, step);
  return hipGetLastError();
}

template <typename T>
__global__ void copy_kernel(const T *__restrict__ x, T *__restrict__ y, size_t n)
{
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) y[i] = x[i];
}

template <typename T>
hipError_t launch_copy(const T *x, T *y, size_t n, hipStream_t s)
{
  copy_kernel<T><<<2048, 256, 0, s>>>(x, y, n);
  return hipGetLastError();
}

template <typename T>
__global__ void mul_kernel(const T *__restrict__ x, const T *__restrict__ k, T *__restrict__ y, size_t n)
{
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    y[i] = x[i] * k[i];
}

template <typename T>
hipError_t launch_mul(const T *x, const T *k, T *y, size_t n, hipStream_t s)
{
  mul_kernel<T><<<2048, 256, 0, s>>>(x, k, y, n);
  return hipGetLastError();
}

__global__ void set_kernel(double *dst, double v)
{
  if (threadIdx.x == 0) dst[0] = v;
}

hipError_t launch_set(double *dst, double v, hipStream_t s)
{
  set_kernel<<<1, 64, 0, s>>>(dst, v);
  return hipGetLastError();
}

#define FFPAT_INST(T)                                                                                          \
  template hipError_t launch_sumsq<T>(const T *, size_t, double *, hipStream_t);                              \
  template hipError_t launch_dot<T>(const T *, const T *, size_t, double *, hipStream_t);                     \
  template hipError_t launch_fill<T>(T *, size_t, double, hipStream_t);                                       \
  template hipError_t launch_normalize<T>(const T *, T *, size_t, const double *, hipStream_t);               \
  template hipError_t launch_prox_l2<T>(T *, const T *, size_t, const double *, double, int, const uint8_t *, \
                                        hipStream_t);                                                         \
  template hipError_t launch_grad_step<T>(const T *, const T *, T *, size_t, const double *, hipStream_t);    \
  template hipError_t launch_copy<T>(const T *, T *, size_t, hipStream_t);                                 \
  template hipError_t launch_mul<T>(const T *, const T *, T *, size_t, hipStream_t);
FFPAT_INST(float)
FFPAT_INST(double)
#undef FFPAT_INST

}  // namespace ffpat

// ===========================================================================
// Gradient regulariser and its prox (conjugate gradients, device scalars).
// ===========================================================================
namespace ffpat {

// (N u) at (x, y, z): 7-point (5-point in 2D) negative Laplacian / dx^2, zero outside.
template <typename T>
__device__ __forceinline__ T neglap_at(const T *__restrict__ u, int x, int y, int z, int nx, int ny, int nz, int ndim,
                                       T inv_dx2)
{
  const size_t sy = (size_t)nx, sz = (size_t)nx * ny;
  const size_t i = (size_t)z * sz + (size_t)y * sy + x;
  const T c = u[i];
  T acc = T(2 * ndim) * c;
  if (x > 0) acc -= u[i - 1];
  if (x + 1 < nx) acc -= u[i + 1];
  if (y > 0) acc -= u[i - sy];
  if (y + 1 < ny) acc -= u[i + sy];
  if (ndim == 3) {
    if (z > 0) acc -= u[i - sz];
    if (z + 1 < nz) acc -= u[i + sz];
  }
  return acc * inv_dx2;
}

__device__ inline double block_sum_256b(double v, double *red)
{
  red[threadIdx.x] = v;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  return red[0];
}

// grid-stride over voxels with (x, y, z) decoded from the linear index
#define FFPAT_VOXEL_LOOP(d, i, x, y, z)                                                                 \
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < (d).nvox();                    \
       i += (size_t)gridDim.x * blockDim.x)                                                          \
    if (int x = (int)(i % (size_t)(d).nx), y = (int)((i / (size_t)(d).nx) % (size_t)(d).ny),         \
        z = (int)(i / ((size_t)(d).nx * (d).ny)); true)

template <typename T>
__global__ void __launch_bounds__(256) neglap_dot_kernel(Dims d, T inv_dx2, const T *__restrict__ h, double *partials)
{
  __shared__ double red[256];
  double acc = 0.0;
  FFPAT_VOXEL_LOOP(d, i, x, y, z) acc += (double)h[i] * (double)neglap_at(h, x, y, z, d.nx, d.ny, d.nz, d.ndim, inv_dx2);
  const double t = block_sum_256b(acc, red);
  if (threadIdx.x == 0) partials[blockIdx.x] = t;
}

template <typename T>
hipError_t launch_neglap_dot(const Dims &d, double dx, const T *h, double *partials, hipStream_t s)
{
  neglap_dot_kernel<T><<<kReduceBlocks, kReduceThreads, 0, s>>>(d, (T)(1.0 / (dx * dx)), h, partials);
  return hipGetLastError();
}

// r = f - (x + tau N x), p = r; partial sums of r.r and f.f
template <typename T>
__global__ void __launch_bounds__(256)
cg_init_kernel(Dims d, T inv_dx2, const T *__restrict__ f, const T *__restrict__ xv, T *__restrict__ r,
               T *__restrict__ p, const double *step, double lambda, double *prr, double *pff)
{
  __shared__ double red[256];
  const T tau = (T)(step[0] * lambda);
  double rr = 0.0, ff = 0.0;
  FFPAT_VOXEL_LOOP(d, i, x, y, z) {
    const T ri = f[i] - (xv[i] + tau * neglap_at(xv, x, y, z, d.nx, d.ny, d.nz, d.ndim, inv_dx2));
    r[i] = ri;
    p[i] = ri;
    rr += (double)ri * (double)ri;
    ff += (double)f[i] * (double)f[i];
  }
  const double a = block_sum_256b(rr, red);
  if (threadIdx.x == 0) prr[blockIdx.x] = a;
  __syncthreads();
  const double b = block_sum_256b(ff, red);
  if (threadIdx.x == 0) pff[blockIdx.x] = b;
}

template <typename T>
hipError_t launch_cg_init(const Dims &d, double dx, const T *f, const T *x, T *r, T *p, const double *step,
                          double lambda, double *partials_rr, double *partials_ff, hipStream_t s)
{
  cg_init_kernel<T><<<kReduceBlocks, kReduceThreads, 0, s>>>(d, (T)(1.0 / (dx * dx)), f, x, r, p, step, lambda,
                                                              partials_rr, partials_ff);
  return hipGetLastError();
}

// q = p + tau N p; partial sums of p.q
template <typename T>
__global__ void __launch_bounds__(256)
cg_apply_kernel(Dims d, T inv_dx2, const T *__restrict__ p, T *__restrict__ q, const double *step, double lambda,
                const double *cg, double *partials)
{
  __shared__ double red[256];
  if (cg[6] != 0.0) return;
  const T tau = (T)(step[0] * lambda);
  double acc = 0.0;
  FFPAT_VOXEL_LOOP(d, i, x, y, z) {
    const T qi = p[i] + tau * neglap_at(p, x, y, z, d.nx, d.ny, d.nz, d.ndim, inv_dx2);
    q[i] = qi;
    acc += (double)p[i] * (double)qi;
  }
  const double t = block_sum_256b(acc, red);
  if (threadIdx.x == 0) partials[blockIdx.x] = t;
}

template <typename T>
hipError_t launch_cg_apply(const Dims &d, double dx, const T *p, T *q, const double *step, double lambda,
                           const double *cg, double *partials, hipStream_t s)
{
  cg_apply_kernel<T><<<kReduceBlocks, kReduceThreads, 0, s>>>(d, (T)(1.0 / (dx * dx)), p, q, step, lambda, cg,
                                                               partials);
  return hipGetLastError();
}

// x += alpha p; r -= alpha q; partial sums of r.r
template <typename T>
__global__ void __launch_bounds__(256)
cg_update_kernel(size_t n, T *__restrict__ xv, T *__restrict__ r, const T *__restrict__ p, const T *__restrict__ q,
                 const double *cg, double *partials)
{
  __shared__ double red[256];
  if (cg[6] != 0.0) return;
  const T alpha = (T)cg[4];
  double acc = 0.0;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
    xv[i] += alpha * p[i];
    const T ri = r[i] - alpha * q[i];
    r[i] = ri;
    acc += (double)ri * (double)ri;
  }
  const double t = block_sum_256b(acc, red);
  if (threadIdx.x == 0) partials[blockIdx.x] = t;
}

template <typename T>
hipError_t launch_cg_update(const Dims &d, T *x, T *r, const T *p, const T *q, const double *cg, double *partials,
                            hipStream_t s)
{
  cg_update_kernel<T><<<kReduceBlocks, kReduceThreads, 0, s>>>(d.nvox(), x, r, p, q, cg, partials);
  return hipGetLastError();
}

// p = r + beta p (cg[5] is beta of the step just finished; skipped once converged)
template <typename T>
__global__ void cg_direction_kernel(size_t n, T *__restrict__ p, const T *__restrict__ r, const double *cg)
{
  if (cg[6] != 0.0) return;
  const T beta = (T)cg[5];
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    p[i] = r[i] + beta * p[i];
}

template <typename T>
hipError_t launch_cg_direction(const Dims &d, T *p, const T *r, const double *cg, hipStream_t s)
{
  cg_direction_kernel<T><<<2048, 256, 0, s>>>(d.nvox(), p, r, cg);
  return hipGetLastError();
}

__global__ void cg_check_init_kernel(double *cg, double tol)
{
  if (threadIdx.x == 0) {
    cg[7] = 0.0;
    cg[6] = (cg[0] <= tol * tol * cg[1]) ? 1.0 : 0.0;
  }
}

__global__ void cg_alpha_kernel(double *cg)
{
  if (threadIdx.x == 0 && cg[6] == 0.0) cg[4] = cg[2] != 0.0 ? cg[0] / cg[2] : 0.0;
}

__global__ void cg_beta_kernel(double *cg, double tol)
{
  if (threadIdx.x == 0 && cg[6] == 0.0) {
    cg[5] = cg[0] != 0.0 ? cg[3] / cg[0] : 0.0;
    cg[0] = cg[3];
    cg[7] += 1.0;
    if (cg[3] <= tol * tol * cg[1] || !isfinite(cg[3])) cg[6] = 1.0;
  }
}

hipError_t launch_cg_check_init(double *cg, double tol, hipStream_t s)
{
  cg_check_init_kernel<<<1, 64, 0, s>>>(cg, tol);
  return hipGetLastError();
}
hipError_t launch_cg_alpha(double *cg, hipStream_t s)
{
  cg_alpha_kernel<<<1, 64, 0, s>>>(cg);
  return hipGetLastError();
}
hipError_t launch_cg_beta(double *cg, double tol, hipStream_t s)
{
  cg_beta_kernel<<<1, 64, 0, s>>>(cg, tol);
  return hipGetLastError();
}

template <typename T>
__global__ void apply_support_kernel(T *h, const uint8_t *__restrict__ support, size_t n)
{
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    if (!support[i]) h[i] = T(0);
}

template <typename T>
hipError_t launch_apply_support(T *h, const uint8_t *support, size_t n, hipStream_t s)
{
  apply_support_kernel<T><<<2048, 256, 0, s>>>(h, support, n);
  return hipGetLastError();
}

template <typename T>
__global__ void __launch_bounds__(256) vol_residual_kernel(T *w, const T *__restrict__ g, size_t n, double *partials)
{
  __shared__ double red[256];
  double acc = 0.0;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
    const T r = w[i] - g[i];
    w[i] = r;
    acc += (double)r * (double)r;
  }
  const double t = block_sum_256b(acc, red);
  if (threadIdx.x == 0) partials[blockIdx.x] = t;
}

template <typename T>
hipError_t launch_vol_residual(T *w, const T *g, size_t n, double *partials, hipStream_t s)
{
  vol_residual_kernel<T><<<kReduceBlocks, kReduceThreads, 0, s>>>(w, g, n, partials);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// The gradient regulariser's prox solved directly (3D).  With zero values outside
// the grid, the 7-point operator N is a sum over the axes of the 1D operator
// (2 u_j - u_{j-1} - u_{j+1}) / dx^2, which the sine transform DST-I diagonalises:
// S_kj = sin(pi (k+1)(j+1) / (n+1)) is symmetric with S S = (n+1)/2 I and
// eigenvalues mu_k = (2 - 2 cos(pi (k+1) / (n+1))) / dx^2.  Hence
// (I + tau N)^{-1} f = S3 D S3 f, S3 = S_x S_y S_z (one transform per axis) and
// D = 8 / ((nx+1)(ny+1)(nz+1)) / (1 + tau (mu_x + mu_y + mu_z)): six transforms
// and one scaling, exact up to rounding.
// Tables (in a volume buffer of at least nx^2 + ny^2 + nz^2 + nx + ny + nz
// elements): S_x, S_y, S_z row-major, then mu_x, mu_y, mu_z.
// ---------------------------------------------------------------------------
template <typename T>
__global__ void dst_tables_kernel(T *tab, int nx, int ny, int nz, double inv_dx2)
{
  const long sx = (long)nx * nx, sy = (long)ny * ny, sz = (long)nz * nz;
  const long total = sx + sy + sz + nx + ny + nz;
  for (long e = (long)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (long)gridDim.x * blockDim.x) {
    long r = e;
    if (r < sx + sy + sz) {
      int n = nx;
      if (r >= sx) {
        r -= sx;
        n = ny;
        if (r >= sy) {
          r -= sy;
          n = nz;
        }
      }
      const long k = r / n, j = r - k * n;
      const long m = ((k + 1) * (j + 1)) % (2L * (n + 1));   // exact argument reduction
      tab[e] = (T)sinpi((double)m / (double)(n + 1));
    } else {
      r -= sx + sy + sz;
      int n = nx;
      if (r >= nx) {
        r -= nx;
        n = ny;
        if (r >= ny) {
          r -= ny;
          n = nz;
        }
      }
      tab[e] = (T)((2.0 - 2.0 * cospi((double)(r + 1) / (double)(n + 1))) * inv_dx2);
    }
  }
}

template <typename T>
hipError_t launch_dst_tables(const Dims &d, double dx, T *tab, hipStream_t s)
{
  dst_tables_kernel<T><<<256, 256, 0, s>>>(tab, d.nx, d.ny, d.nz, 1.0 / (dx * dx));
  return hipGetLastError();
}

// out = S in along one axis.  The volume is viewed as [A][n][B] (B = 1 for x, nx for
// y, nx ny for z); column c = a B + b holds the n values at a n B + b + j B.  A
// work-group takes 64 columns and every k, in tiles of 64 (16 per thread, the
// thread's column fixed); j runs in chunks of 32 through LDS (the columns' values and
// the transposed S tile), zero-filled beyond n and beyond the last column.
template <typename T>
__global__ void __launch_bounds__(256)
dst_axis_kernel(const T *__restrict__ in, T *__restrict__ out, const T *__restrict__ S, int n, long B, long ncols)
{
  constexpr int CT = 64, JC = 32, KT = 64, KP = KT + 4;
  __shared__ T X[JC][CT + 1];
  __shared__ __attribute__((aligned(16))) T St[JC][KP];
  const int tid = threadIdx.x, col = tid & 63, kg = tid >> 6;
  const long c0 = (long)blockIdx.x * CT;
  const long cme = c0 + col;
  const bool cin = cme < ncols;
  long bme = 0;                               // offset of this thread's column (B > 1)
  if (cin) {
    const long a = cme / B;
    bme = a * (long)n * B + (cme - a * B);
  }
  for (int k0 = 0; k0 < n; k0 += KT) {
    T acc[16];
#pragma unroll
    for (int q = 0; q < 16; ++q) acc[q] = T(0);
    for (int j0 = 0; j0 < n; j0 += JC) {
      __syncthreads();                        // the previous chunk's tiles are read
      if (B == 1) {                           // x: each line contiguous, lanes along j
#pragma unroll
        for (int i = 0; i < 8; ++i) {
          const int cc = (tid >> 5) + 8 * i, jj = tid & 31;
          const long c = c0 + cc;
          const int j = j0 + jj;
          X[jj][cc] = (c < ncols && j < n) ? in[c * n + j] : T(0);
        }
      } else {                                // y, z: lanes along the columns
#pragma unroll
        for (int i = 0; i < 8; ++i) {
          const int jj = (tid >> 6) + 4 * i;
          const int j = j0 + jj;
          X[jj][col] = (cin && j < n) ? in[bme + (long)j * B] : T(0);
        }
      }
#pragma unroll
      for (int i = 0; i < 8; ++i) {
        const int e = tid + 256 * i, kk = e >> 5, jj = e & 31;
        const int k = k0 + kk, j = j0 + jj;
        St[jj][kk] = (k < n && j < n) ? S[(long)k * n + j] : T(0);
      }
      __syncthreads();
#pragma unroll 4
      for (int jj = 0; jj < JC; ++jj) {
        const T x = X[jj][col];
#pragma unroll
        for (int q = 0; q < 16; ++q) acc[q] += St[jj][kg * 16 + q] * x;
      }
    }
    if (cin) {
#pragma unroll
      for (int q = 0; q < 16; ++q) {
        const int k = k0 + kg * 16 + q;
        if (k < n) out[(B == 1 ? cme * n : bme) + (long)k * B] = acc[q];
      }
    }
  }
}

template <typename T>
hipError_t launch_dst_axis(const Dims &d, int axis, const T *in, T *out, const T *S, hipStream_t s)
{
  const int n = axis == 0 ? d.nx : axis == 1 ? d.ny : d.nz;
  const long B = axis == 0 ? 1L : axis == 1 ? (long)d.nx : (long)d.nx * d.ny;
  const long ncols = (long)d.nvox() / n;
  const long groups = (ncols + 63) / 64;
  if (groups > 0x7fffffffL) return hipErrorInvalidValue;
  dst_axis_kernel<T><<<(unsigned)groups, 256, 0, s>>>(in, out, S, n, B, ncols);
  return hipGetLastError();
}

// u *= 8 / ((nx+1)(ny+1)(nz+1)) / (1 + step lambda (mu_x + mu_y + mu_z))
template <typename T>
__global__ void dst_scale_kernel(T *u, Dims d, const T *mu, const double *step, double lambda)
{
  const double tau = step[0] * lambda;
  const double norm = 8.0 / (((double)d.nx + 1.0) * ((double)d.ny + 1.0) * ((double)d.nz + 1.0));
  const T *mx = mu, *my = mu + d.nx, *mz = mu + d.nx + d.ny;
  FFPAT_VOXEL_LOOP(d, i, x, y, z) {
    const double den = 1.0 + tau * ((double)mx[x] + (double)my[y] + (double)mz[z]);
    u[i] = (T)((double)u[i] * (norm / den));
  }
}

template <typename T>
hipError_t launch_dst_scale(const Dims &d, T *u, const T *mu, const double *step, double lambda, hipStream_t s)
{
  dst_scale_kernel<T><<<2048, 256, 0, s>>>(u, d, mu, step, lambda);
  return hipGetLastError();
}

#define FFPAT_INST2(T)                                                                                          \
  template hipError_t launch_neglap_dot<T>(const Dims &, double, const T *, double *, hipStream_t);              \
  template hipError_t launch_cg_init<T>(const Dims &, double, const T *, const T *, T *, T *, const double *,     \
                                        double, double *, double *, hipStream_t);                              \
  template hipError_t launch_cg_apply<T>(const Dims &, double, const T *, T *, const double *, double,          \
                                         const double *, double *, hipStream_t);                               \
  template hipError_t launch_cg_update<T>(const Dims &, T *, T *, const T *, const T *, const double *, double *, \
                                          hipStream_t);                                                        \
  template hipError_t launch_cg_direction<T>(const Dims &, T *, const T *, const double *, hipStream_t);        \
  template hipError_t launch_dst_tables<T>(const Dims &, double, T *, hipStream_t);                          \
  template hipError_t launch_dst_axis<T>(const Dims &, int, const T *, T *, const T *, hipStream_t);          \
  template hipError_t launch_dst_scale<T>(const Dims &, T *, const T *, const double *, double, hipStream_t); \
  template hipError_t launch_apply_support<T>(T *, const uint8_t *, size_t, hipStream_t);                       \
  template hipError_t launch_vol_residual<T>(T *, const T *, size_t, double *, hipStream_t);
FFPAT_INST2(float)
FFPAT_INST2(double)
#undef FFPAT_INST2

}  // namespace ffpat
