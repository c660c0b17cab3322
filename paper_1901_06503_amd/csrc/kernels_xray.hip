// Plane-wise X-ray transform X (eq. Radon, Sec. 2.1), its transpose (the
// backprojection of Sec. 3.1) and the ramp preconditioner Lambda (Sec. 3.1).
//
// X uses linear interpolation along the minor axis of each ray (Sec. 4.1
// names linear interpolation).  The projector walks the ray one grid line
// of the major axis at a time (Joseph's method); the backprojector gathers
// the same weights per voxel, so the two are exact transposes.
#include "kernels.h"

namespace ffpat {

// ---------------------------------------------------------------------------
// Projector: one thread per detector bin (a, z, j), coalesced writes along s.
// ---------------------------------------------------------------------------
template <typename T>
__global__ void __launch_bounds__(256)
project_kernel(const T *__restrict__ vol, T *__restrict__ g, const AngleParams *__restrict__ ap, int nx, int ny,
               int nz, int ns)
{
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  const int z = blockIdx.y;
  const int a = blockIdx.z;
  if (j >= ns) return;
  const AngleParams P = ap[a];
  const T *plane = vol + (size_t)z * nx * ny;
  int nr, nm;
  size_t sr, sm;
  if (P.major_x) {  // march over columns x_r, interpolate along y
    nr = nx; nm = ny; sr = 1; sm = (size_t)nx;
  } else {          // march over rows y_r, interpolate along x
    nr = ny; nm = nx; sr = (size_t)nx; sm = 1;
  }
  const double A = P.u0 + (double)j * P.uj;
  // marched lines whose crossing u lies in (-1, nm), where a tap can be inside
  double lo = 0.0, hi = (double)(nr - 1);
  if (P.ur != 0.0) {
    double r_a = (-1.0 - A) / P.ur, r_b = ((double)nm - A) / P.ur;
    if (r_a > r_b) { double t = r_a; r_a = r_b; r_b = t; }
    lo = fmin(fmax(lo, floor(r_a)), (double)nr);   // clamped before any int conversion
    hi = fmax(fmin(hi, ceil(r_b)), -1.0);
  } else if (!(A > -1.0 && A < (double)nm)) {
    hi = -1.0;
  }
  T acc = T(0);
  for (int r = (int)lo; r <= (int)hi; ++r) {
    const double u = fma((double)r, P.ur, A);
    const double fl = floor(u);
    const int i0 = (int)fl;
    const T f = (T)(u - fl);
    const T *line = plane + (size_t)r * sr;
    const T v0 = (i0 >= 0 && i0 < nm) ? line[(size_t)i0 * sm] : T(0);
    const T v1 = (i0 + 1 >= 0 && i0 + 1 < nm) ? line[(size_t)(i0 + 1) * sm] : T(0);
    acc += (T(1) - f) * v0 + f * v1;
  }
  g[((size_t)a * nz + z) * ns + j] = acc * (T)P.w;
}

template <typename T>
hipError_t launch_project(const Dims &d, int n_angles, int ns, const AngleParams *ap, const T *vol, T *g,
                          hipStream_t s)
{
  const int tb = ns >= 256 ? 256 : ((ns + 63) / 64) * 64;
  dim3 grid((ns + tb - 1) / tb, d.nz, n_angles);
  project_kernel<T><<<grid, tb, 0, s>>>(vol, g, ap, d.nx, d.ny, d.nz, ns);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Backprojector: one thread per voxel, loop over angles, <= 2 taps per angle
// when ds = dx (the footprint half-width m dx / ds is at most one bin).
// ---------------------------------------------------------------------------
template <typename T>
__global__ void __launch_bounds__(256)
backproject_kernel(const T *__restrict__ g, T *__restrict__ vol, const AngleParams *__restrict__ ap, int n_angles,
                   int nx, int ny, int nz, int ns, const T *__restrict__ kap)
{
  const int i = blockIdx.x * 64 + threadIdx.x;
  const int k = blockIdx.y * 4 + threadIdx.y;
  const int z = blockIdx.z;
  if (i >= nx || k >= ny) return;
  T acc = T(0);
  for (int a = 0; a < n_angles; ++a) {
    const AngleParams &P = ap[a];
    const double t = P.b0 + (double)i * P.bi + (double)k * P.bk;
    const T *row = g + ((size_t)a * nz + z) * ns;
    const int jlo = (int)fmin(fmax(ceil(t - P.hw), 0.0), (double)ns);
    const int jhi = (int)fmax(fmin(floor(t + P.hw), (double)(ns - 1)), -1.0);
    T sum = T(0);
    for (int j = jlo; j <= jhi; ++j) {
      const double wt = 1.0 - fabs((double)j - t) * P.inv_hw;
      if (wt > 0.0) sum += (T)wt * row[j];
    }
    acc += sum * (T)P.w;
  }
  const size_t idx = ((size_t)z * ny + k) * nx + i;
  vol[idx] = kap ? acc * kap[idx] : acc;
}

template <typename T>
hipError_t launch_backproject(const Dims &d, int n_angles, int ns, const AngleParams *ap, const T *g, T *vol,
                              const T *kap, hipStream_t s)
{
  dim3 block(64, 4, 1);
  dim3 grid((d.nx + 63) / 64, (d.ny + 3) / 4, d.nz);
  backproject_kernel<T><<<grid, block, 0, s>>>(g, vol, ap, n_angles, d.nx, d.ny, d.nz, ns, kap);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Residual + ramp filter: one work-group per detector row (a, z).
//   r = mask (g - G);  y = mask (taps * r)  (Toeplitz, taps[n] = C h_n);
//   row_partials[row] = sum_j r_j y_j  (FP64, fixed-order tree).
// ---------------------------------------------------------------------------
template <typename T>
__global__ void __launch_bounds__(256)
residual_ramp_kernel(const T *g, const T *__restrict__ G, const uint8_t *__restrict__ mask,
                     const T *__restrict__ taps, T *y, int ns, double *row_partials)
{
  extern __shared__ unsigned char smem_raw[];
  T *r = reinterpret_cast<T *>(smem_raw);
  __shared__ double red[256];
  const size_t row = blockIdx.x;
  const size_t base = row * (size_t)ns;
  for (int j = threadIdx.x; j < ns; j += blockDim.x) {
    T v = g[base + j];
    if (G) v -= G[base + j];
    if (mask && !mask[base + j]) v = T(0);
    r[j] = v;
  }
  __syncthreads();
  double part = 0.0;
  for (int j = threadIdx.x; j < ns; j += blockDim.x) {
    T acc;
    if (taps) {
      acc = taps[0] * r[j];
      for (int n = 1; n < ns; n += 2) {
        T pair = T(0);
        if (j - n >= 0) pair += r[j - n];
        if (j + n < ns) pair += r[j + n];
        acc += taps[n] * pair;
      }
    } else {
      acc = r[j];
    }
    if (mask && !mask[base + j]) acc = T(0);
    y[base + j] = acc;
    part += (double)r[j] * (double)acc;
  }
  if (row_partials) {
    red[threadIdx.x] = part;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
      if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
      __syncthreads();
    }
    if (threadIdx.x == 0) row_partials[row] = red[0];
  }
}

template <typename T>
hipError_t launch_residual_ramp(int rows, int ns, const T *g, const T *G, const uint8_t *mask, const T *taps, T *y,
                                double *row_partials, hipStream_t s)
{
  const size_t shmem = (size_t)ns * sizeof(T);
  residual_ramp_kernel<T><<<rows, 256, shmem, s>>>(g, G, mask, taps, y, ns, row_partials);
  return hipGetLastError();
}

#define FFPAT_INST(T)                                                                                         \
  template hipError_t launch_project<T>(const Dims &, int, int, const AngleParams *, const T *, T *,         \
                                        hipStream_t);                                                        \
  template hipError_t launch_backproject<T>(const Dims &, int, int, const AngleParams *, const T *, T *,     \
                                            const T *, hipStream_t);                                         \
  template hipError_t launch_residual_ramp<T>(int, int, const T *, const T *, const uint8_t *, const T *, T *, \
                                              double *, hipStream_t);
FFPAT_INST(float)
FFPAT_INST(double)
#undef FFPAT_INST

}  // namespace ffpat
