// Shared pieces of the e2m1 (FP4) sweep kernels (sweep_mfma4.hip, couplings
// in LDS; sweep_big4.hip, couplings streamed): the matrix-core call, the
// spin encodings and their conversions.
//
// Spins enter the matrix unit as e2m1 +-2.0 (s = +1 -> 0x4, s = -1 -> 0xC):
// the top two bits of a nibble, read as a signed 2-bit field, are s itself.
// A lane's 16 spins r = 0..15 of a row tile (spin 32 mt + 16 half + r) sit in
// two words q = 0, 1: byte b of word q holds spin 8q + b in its low nibble
// and spin 8q + 4 + b in its high nibble -- the order pack_f4_fragments packs
// J's K dimension in.  As int8 (+-1 bytes, the layout of stored states) they
// sit in four words k: byte b of word k is spin 4k + b.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace pim {
namespace e2m1 {

typedef int v4i __attribute__((ext_vector_type(4)));
typedef int v8i __attribute__((ext_vector_type(8)));
typedef float v16f __attribute__((ext_vector_type(16)));

constexpr uint32_t kPlusTwos = 0x44444444u;   // eight e2m1 +2.0 (sign bit 3 of each nibble clear)
constexpr int kTab32Bytes = kTabEntries * 4;  // a step table in LDS: 512 doubled thresholds, 32-bit

// C += A . B on 32x64 / 64x32 e2m1 operands (16 bytes per lane; the upper
// half of the 8-register operand is unused for this format).  Zero scale
// operands select the unscaled instruction.
__device__ __forceinline__ v16f mfma(v4i a, v4i b, v16f c) {
  const v8i a8 = {a[0], a[1], a[2], a[3], 0, 0, 0, 0};
  const v8i b8 = {b[0], b[1], b[2], b[3], 0, 0, 0, 0};
  return __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(a8, b8, c, 4, 4, 0, 0, 0, 0);
}

// int8 spins of rows 8q..8q+3 (lo) and 8q+4..8q+7 (hi) -> one e2m1 word
__device__ __forceinline__ uint32_t nib_from_i8(uint32_t lo, uint32_t hi) {
  return ((lo >> 4) & 0x08080808u) | (hi & 0x80808080u) | kPlusTwos;
}
// e2m1 word -> int8 spins of rows 8q + 4 hi + b, b = 0..3
__device__ __forceinline__ uint32_t i8_from_nib(uint32_t w, int hi) {
  return 0x01010101u + 0xFEu * ((w >> (4 * hi + 3)) & 0x01010101u);
}
// a lane's two e2m1 words of a tile -> its 16 int8 spins
__device__ __forceinline__ v4i i8_tile(uint2 w) {
  return v4i{(int)i8_from_nib(w.x, 0), (int)i8_from_nib(w.x, 1), (int)i8_from_nib(w.y, 0),
             (int)i8_from_nib(w.y, 1)};
}
// the four int8 words of s(0) -> the tile's two e2m1 words
__device__ __forceinline__ uint2 nib_tile(v4i v) {
  return uint2{nib_from_i8((uint32_t)v[0], (uint32_t)v[1]), nib_from_i8((uint32_t)v[2], (uint32_t)v[3])};
}
// S2 initial spins: +1 where the byte's top bit (u >= 128) is set, -1
// elsewhere (int8)
__device__ __forceinline__ uint32_t spins_from_bits(uint32_t w) {
  return 0xFFFFFFFFu - 0xFEu * ((w >> 7) & 0x01010101u);
}
// s of register r of a tile, from its two e2m1 words: +1 / -1
__device__ __forceinline__ int spin_of(const uint32_t (&sw)[2], int r) {
  return (int)__builtin_amdgcn_sbfe(sw[r >> 3], 8 * (r & 3) + 4 * ((r >> 2) & 1) + 2, 2);
}

}  // namespace e2m1
}  // namespace pim
