// Copy of host inputs (batch plans, shear points) from the handle's pinned,
// device-mapped staging buffer into device workspace.  A kernel rather than
// an asynchronous memory copy, so that a call captured into a graph records
// kernel nodes only.  Source and destination are 16-byte aligned; the byte
// count is a multiple of 4 (the pieces are int32, int64 and double arrays).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>

namespace bsi {

namespace {

__global__ void __launch_bounds__(256) stage_copy_kernel(const uint4* __restrict__ src,
                                                         uint4* __restrict__ dst, int64_t n16,
                                                         int tail_words) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n16; i += stride) dst[i] = src[i];
  if (blockIdx.x == 0 && (int)threadIdx.x < tail_words)
    reinterpret_cast<uint32_t*>(dst + n16)[threadIdx.x] =
        reinterpret_cast<const uint32_t*>(src + n16)[threadIdx.x];
}

}  // namespace

hipError_t launch_stage_copy(const void* src_dev, void* dst, size_t bytes, hipStream_t s) {
  if (bytes == 0) return hipSuccess;
  if ((bytes & 3) || (reinterpret_cast<uintptr_t>(src_dev) & 15) || (reinterpret_cast<uintptr_t>(dst) & 15))
    return hipErrorInvalidValue;
  const int64_t n16 = (int64_t)(bytes / 16);
  const int tail = (int)((bytes % 16) / 4);
  const int64_t blocks = std::min<int64_t>(std::max<int64_t>((n16 + 255) / 256, 1), 1024);
  hipLaunchKernelGGL(stage_copy_kernel, dim3((unsigned)blocks), dim3(256), 0, s,
                     static_cast<const uint4*>(src_dev), static_cast<uint4*>(dst), n16, tail);
  return hipGetLastError();
}

}  // namespace bsi
