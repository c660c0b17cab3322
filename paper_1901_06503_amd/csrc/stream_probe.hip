// Streaming ceilings for the roofline of the leapfrog kernels, built as its own
// library (libffpat_probe.so) for the benchmark; not part of the method's C ABI.
//
// Two plain element-wise kernels with 16-byte accesses and a grid-stride loop:
//   pattern 0: the access pattern of the two-step stencil: three fields read and two
//              written, each element once (a leapfrog-like update, so that nothing
//              can be elided);
//   pattern 1: a copy, one field read and one written.
// What they reach on a device bounds what a kernel with the same streams can reach
// there, for fields of the same size.
#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

namespace ffpat_probe {

__global__ void __launch_bounds__(256)
read3_write2(const float4 *__restrict__ a, const float4 *__restrict__ b, const float4 *__restrict__ c,
             float4 *__restrict__ q, float4 *__restrict__ o, size_t n4)
{
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n4; i += (size_t)gridDim.x * blockDim.x) {
    const float4 x = a[i], y = b[i], k = c[i];
    float4 u, v;
    u.x = 2.f * y.x - x.x + k.x * y.x;
    u.y = 2.f * y.y - x.y + k.y * y.y;
    u.z = 2.f * y.z - x.z + k.z * y.z;
    u.w = 2.f * y.w - x.w + k.w * y.w;
    v.x = 2.f * u.x - y.x + k.x * u.x;
    v.y = 2.f * u.y - y.y + k.y * u.y;
    v.z = 2.f * u.z - y.z + k.z * u.z;
    v.w = 2.f * u.w - y.w + k.w * u.w;
    q[i] = u;
    o[i] = v;
  }
}

__global__ void __launch_bounds__(256)
read1_write1(const float4 *__restrict__ a, float4 *__restrict__ q, size_t n4)
{
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n4; i += (size_t)gridDim.x * blockDim.x)
    q[i] = a[i];
}

bool aligned16(const void *p) { return p && ((uintptr_t)p & 15) == 0; }

}  // namespace ffpat_probe

using namespace ffpat_probe;

// One launch of `pattern` over fields of n_floats floats (a multiple of 4; every
// pointer a 16-byte aligned device buffer of that size; pattern 1 uses a and q only)
// with `blocks` work-groups of 256 threads on `stream`.  Returns 0, -1 for a bad
// argument (nothing launched), -4 if the launch failed.
extern "C" int ffpat_probe_stream(int pattern, const void *a, const void *b, const void *c, void *q, void *o,
                                  size_t n_floats, int blocks, void *stream)
{
  if (n_floats == 0 || n_floats % 4 != 0 || blocks < 1 || !aligned16(a) || !aligned16(q)) return -1;
  const hipStream_t s = static_cast<hipStream_t>(stream);
  const size_t n4 = n_floats / 4;
  if (pattern == 0) {
    if (!aligned16(b) || !aligned16(c) || !aligned16(o)) return -1;
    read3_write2<<<blocks, 256, 0, s>>>(static_cast<const float4 *>(a), static_cast<const float4 *>(b),
                                        static_cast<const float4 *>(c), static_cast<float4 *>(q),
                                        static_cast<float4 *>(o), n4);
  } else if (pattern == 1) {
    read1_write1<<<blocks, 256, 0, s>>>(static_cast<const float4 *>(a), static_cast<float4 *>(q), n4);
  } else {
    return -1;
  }
  return hipGetLastError() == hipSuccess ? 0 : -4;
}
