// Measurement helpers: the reference read + write stream that the
// collide-stream kernel's HBM fraction is compared with (ib_lbm_stream_copy).
#include "ib_lbm_internal.h"

namespace iblbm {

// 16 bytes per thread and round, grid-stride.
__global__ __launch_bounds__(1024) void stream_copy_kernel(const float4 *__restrict__ a,
                                                           float4 *__restrict__ b, size_t n) {
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += stride) b[i] = a[i];
}

hipError_t launch_stream_copy(const void *src, void *dst, size_t n, int workgroups, hipStream_t stream) {
  hipLaunchKernelGGL(stream_copy_kernel, dim3(workgroups), dim3(1024), 0, stream, (const float4 *)src,
                     (float4 *)dst, n);
  return hipGetLastError();
}

}  // namespace iblbm
