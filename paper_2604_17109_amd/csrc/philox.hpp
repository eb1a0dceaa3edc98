// Philox4x32-10 for device code (Salmon, Moraes, Dror, Shaw, "Parallel Random
// Numbers: As Easy as 1, 2, 3", SC'11): ten rounds of the Philox-4x32 S-box
// with multipliers 0xD2511F53 / 0xCD9E8D57 and Weyl key increments
// 0x9E3779B9 / 0xBB67AE85.  Keys are wave-uniform (seed), so the key schedule
// stays in scalar registers; the counter is per lane.
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>

namespace pim {

struct Ctr4 {
  uint32_t x, y, z, w;
};

__device__ __forceinline__ Ctr4 philox4x32_10(Ctr4 c, uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const uint64_t p0 = (uint64_t)0xD2511F53u * c.x;
    const uint64_t p1 = (uint64_t)0xCD9E8D57u * c.z;
    const uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    const uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    // three-way XORs as single v_bitop3_b32 (truth table 0x96 = a ^ b ^ c)
    c = Ctr4{(uint32_t)__builtin_amdgcn_bitop3_b32(hi1, c.y, k0, 0x96), lo1,
             (uint32_t)__builtin_amdgcn_bitop3_b32(hi0, c.w, k1, 0x96), lo0};
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
  return c;
}

// Counter word 3 layout: (domain << 24) | stream id.
constexpr uint32_t kDomainNoise = 0u;
constexpr uint32_t kDomainInit = 1u;

}  // namespace pim
