// stage.hip -- device side of the host stage's check of the vertices a pass
// would attempt: their values and their in-neighbours' values gathered into
// a short buffer, so the host reads kilobytes instead of the whole value
// array when the list is short; a short push's lowered values written back
// the same way.
#include <hip/hip_runtime.h>

#include "engine.hpp"

namespace sr {

namespace {
__global__ void __launch_bounds__(256) gather_u32_kernel(const uint32_t *src, const uint32_t *idx, uint32_t count,
                                                         uint32_t *dst) {
  const uint32_t i = blockIdx.x * 256u + threadIdx.x;
  if (i < count) dst[i] = src[idx[i]];
}

__global__ void __launch_bounds__(256) scatter_u32_kernel(uint32_t *dst, const uint32_t *idx, const uint32_t *vals,
                                                          uint32_t count) {
  const uint32_t i = blockIdx.x * 256u + threadIdx.x;
  if (i < count) dst[idx[i]] = vals[i];
}
}  // namespace

hipError_t launch_gather_u32(const uint32_t *src, const uint32_t *idx, uint32_t count, uint32_t *dst,
                             hipStream_t s) {
  if (count == 0) return hipSuccess;
  hipLaunchKernelGGL(gather_u32_kernel, dim3((count + 255u) / 256u), dim3(256), 0, s, src, idx, count, dst);
  return hipGetLastError();
}

hipError_t launch_scatter_u32(uint32_t *dst, const uint32_t *idx, const uint32_t *vals, uint32_t count,
                              hipStream_t s) {
  if (count == 0) return hipSuccess;
  hipLaunchKernelGGL(scatter_u32_kernel, dim3((count + 255u) / 256u), dim3(256), 0, s, dst, idx, vals, count);
  return hipGetLastError();
}

}  // namespace sr
