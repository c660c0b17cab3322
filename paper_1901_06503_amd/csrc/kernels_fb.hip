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
