// Plain device copy: the reference kernel of known traffic against which the
// hardware byte counters (rocprofv3 FETCH_SIZE / WRITE_SIZE) are scaled.  It
// moves data the way the tile kernels stream their chunks: one dword per lane
// per load instruction, consecutive lanes on consecutive addresses.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "cellmech.h"
#include "handle.h"

namespace cm {
namespace {

constexpr int kCopyThreads = 256;

__global__ __launch_bounds__(kCopyThreads) void stream_copy_kernel(const float* src,
                                                                  float* dst, int64_t n) {
  const int64_t stride = (int64_t)gridDim.x * kCopyThreads;
  for (int64_t i = (int64_t)blockIdx.x * kCopyThreads + threadIdx.x; i < n; i += stride)
    dst[i] = src[i];
}

}  // namespace
}  // namespace cm

extern "C" int cm_stream_copy(const float* src, float* dst, int64_t n, hipStream_t stream) {
  if (n < 0) return cm::api_fail(CM_EINVAL, "n must be >= 0");
  if (n == 0) return CM_OK;
  if (!src || !dst) return cm::api_fail(CM_EINVAL, "src and dst must be device pointers");
  const int64_t blocks = (n + cm::kCopyThreads - 1) / cm::kCopyThreads;
  const unsigned grid = (unsigned)(blocks < 65536 ? blocks : 65536);
  hipLaunchKernelGGL(cm::stream_copy_kernel, dim3(grid), dim3(cm::kCopyThreads), 0, stream, src, dst, n);
  CM_HIP(hipGetLastError());
  return CM_OK;
}
