// Byte copies between device memory and pinned, device-mapped host memory,
// done by a kernel on the caller's stream.  The request server moves a MIMO
// chunk's staged inputs and its results this way: every step of a chunk then
// runs in order on one compute queue, with no hand-off to a copy engine
// between them.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>

#include "internal.hpp"

namespace pim {
namespace {

constexpr int kCopyThreads = 256;
constexpr size_t kCopyMaxBlocks = 1024;

// 16-byte words first (grid-stride), then the tail bytes in block 0
__global__ __launch_bounds__(kCopyThreads) void copy_bytes_kernel(uint8_t* dst, const uint8_t* src, size_t words,
                                                                  size_t bytes) {
  const uint4* s = reinterpret_cast<const uint4*>(src);
  uint4* d = reinterpret_cast<uint4*>(dst);
  const size_t stride = (size_t)gridDim.x * kCopyThreads;
  for (size_t i = (size_t)blockIdx.x * kCopyThreads + threadIdx.x; i < words; i += stride) d[i] = s[i];
  if (blockIdx.x == 0)
    for (size_t i = words * 16 + threadIdx.x; i < bytes; i += kCopyThreads) dst[i] = src[i];
}

}  // namespace

hipError_t launch_copy_bytes(void* dst, const void* src, size_t bytes, hipStream_t s) {
  if (bytes == 0) return hipSuccess;
  if (!dst || !src || (reinterpret_cast<uintptr_t>(dst) | reinterpret_cast<uintptr_t>(src)) % 16)
    return hipErrorInvalidValue;
  const size_t words = bytes / 16;
  const size_t blocks = std::min(kCopyMaxBlocks, std::max<size_t>(1, (words + kCopyThreads - 1) / kCopyThreads));
  hipLaunchKernelGGL(copy_bytes_kernel, dim3((unsigned)blocks), dim3(kCopyThreads), 0, s,
                     static_cast<uint8_t*>(dst), static_cast<const uint8_t*>(src), words, bytes);
  return hipGetLastError();
}

}  // namespace pim
