// A-operand fragments of the streamed sweep kernels (sweep_big.hip, int8;
// sweep_big4.hip, e2m1), read from global memory through a buffer resource.
// Fragment f of an instance is 64 lanes x 16 bytes at byte 1024 f; the
// fragment index is wave-uniform, so its byte offset goes in the scalar
// offset operand and the lane's 16 l in a vector register that never changes.
// A load then needs no vector address arithmetic, where a 64-bit pointer
// costs three vector instructions per load.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace pim {

struct FragStream {
  typedef int v4i __attribute__((ext_vector_type(4)));
  // Buffer descriptor word 3 for gfx9-family raw 32-bit loads (data format 32).
  static constexpr int kRsrcWord3 = 0x00020000;

  __amdgpu_buffer_rsrc_t rsrc;
  int voff;

  // base: fragment 0 of the instance; bytes: the instance's fragment bytes
  // (below 2^31); lane: 0..63.
  __device__ __forceinline__ FragStream(const void* base, uint32_t bytes, int lane)
      : rsrc(__builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), 0, (int)bytes, kRsrcWord3)),
        voff(lane * 16) {}

  // The lane's 16 bytes of fragment f (uniform, 0 <= f < bytes / 1024).
  __device__ __forceinline__ v4i operator()(int f) const {
    return __builtin_amdgcn_raw_buffer_load_b128(rsrc, voff, f * 1024, 0);
  }
};

}  // namespace pim
