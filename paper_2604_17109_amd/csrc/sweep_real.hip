// Persistent PIMI sweep for real-valued couplings on FP8 / BF16 MFMA (gfx950).
//
// Same organisation as the int8 sweep: one workgroup per (instance, up to four
// 32-trial blocks), the instance's quantised couplings staged once in LDS, one
// wave per 32 trials (the MFMA N dimension) holding its spins in registers in
// B-operand layout for the whole run, no barrier inside the step loop.
//
//   I[Npad x 32] = scale * (Q[Npad x Npad] . S[Npad x 32]) + h
//     FP8:  v_mfma_f32_32x32x64_f8f6f4 (OCP e4m3 operands, FP32 accumulation)
//     BF16: v_mfma_f32_32x32x16_bf16
//
// Layout.  Output register r of lane l (column l % 32, half hh = l / 32) holds
// row 8(r/4) + 4hh + r%4, carrying spin 32mt + 16hh + r of row tile mt, as in
// the int8 kernel.  A-slot (hh, p) of a lane pairs with B-slot (hh, p): with
// FP8 (K = 64, 32 slots per half) slot (hh, p) of K step kk carries spin
// 32(2kk + p/16) + 16hh + p%16, i.e. the lane's own 16 spins of row tiles 2kk
// and 2kk+1; with BF16 (K = 16, 8 slots) slot (hh, p) of step (kt, j) carries
// spin 32kt + 16hh + 8j + p.  So new spins go from the accumulator to the next
// step's B operand inside the lane, and a lane-half's 16 spins of a tile are
// one Philox block.  Spins are +-1 encoded in the operand format (FP8 0x38 /
// 0xB8, BF16 0x3F80 / 0xBF80).
//
// Decision.  The host compiles each step into 512 binary32 field thresholds
// over (noise index u, sign of s): s(t+1) = +1 iff I >= tab[u ^ m], m = 0 for
// s = +1 and -1 for s = -1 (relative to the table centre).  I - tab is
// negative exactly when I < tab (also for +-inf thresholds), so its sign bit is
// the new spin's sign.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cmath>
#include <cstdint>
#include <type_traits>

#include "internal.hpp"
#include "philox.hpp"

namespace pim {
namespace {

typedef int v4i __attribute__((ext_vector_type(4)));
typedef int v8i __attribute__((ext_vector_type(8)));
typedef float v16f __attribute__((ext_vector_type(16)));
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));

constexpr int kMaxWaves = 4;
constexpr int kRealTabBytes = kTabEntries * 4;  // 2 KB per step table
// Step tables are fetched this many steps ahead (registers, 8 per step): one
// request's wave is often alone on its SIMD, so a table load issued only one
// step before its use would expose the full memory latency every step.
constexpr int kAhead = 4;
static_assert(kRealTabBytes == 64 * 32, "two 16-byte chunks per lane");

#define PIM_FENCE(v) asm volatile("" : "+v"(v))

// Workgroup barrier for data exchanged through LDS only: each wave waits for
// its own LDS operations, not for its outstanding global loads (prefetches
// stay in flight across it).  A plain __syncthreads() is also a fence for
// global memory and would drain every prefetch at every step.
__device__ __forceinline__ void lds_barrier() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// v4i words per row tile per lane: 16 spins of 1 (FP8) or 2 (BF16) bytes.
template <int PREC> constexpr int words() { return PREC == PIM_PREC_FP8 ? 1 : 2; }

constexpr size_t frag_bytes(int prec, int nt) {
  return prec == PIM_PREC_FP8 ? (size_t)nt * ((nt + 1) / 2) * 2048 : (size_t)nt * nt * 2048;
}

__device__ __forceinline__ uint32_t perm(uint32_t hi, uint32_t lo, uint32_t sel) {
  return __builtin_amdgcn_perm(hi, lo, sel);
}

// int8 spin bytes (+1 = 0x01, -1 = 0xFF) <-> operand encodings
__device__ __forceinline__ uint32_t fp8_from_i8(uint32_t w) { return (w & 0x80808080u) | 0x38383838u; }
__device__ __forceinline__ uint32_t bf16_lo_from_i8(uint32_t w) {  // bytes 0, 1 -> two bf16
  return (perm(w, w, 0x010C000Cu) & 0x80008000u) | 0x3F803F80u;
}
__device__ __forceinline__ uint32_t bf16_hi_from_i8(uint32_t w) {  // bytes 2, 3
  return (perm(w, w, 0x030C020Cu) & 0x80008000u) | 0x3F803F80u;
}
__device__ __forceinline__ uint32_t i8_from_fp8(uint32_t w) { return 0x01010101u + 0xFEu * ((w >> 7) & 0x01010101u); }
__device__ __forceinline__ uint32_t i8_from_bf16(uint32_t w0, uint32_t w1) {
  return perm(w1, w0, 0x0B0A0908u) | 0x01010101u;  // sign bits 15 and 31 of each word
}
__device__ __forceinline__ int spins_from_bits(uint32_t w) {
  return (int)(0xFFFFFFFFu - 0xFEu * ((w >> 7) & 0x01010101u));
}

// 0 for a +1 spin, -1 for a -1 spin: spin r of the lane's 16 in a tile.
template <int PREC>
__device__ __forceinline__ int spin_mask(const uint32_t (&sw)[4 * words<PREC>()], int r) {
  if (PREC == PIM_PREC_FP8) return __builtin_amdgcn_sbfe((int)sw[r >> 2], 8 * (r & 3) + 7, 1);
  return __builtin_amdgcn_sbfe((int)sw[r >> 1], 16 * (r & 1) + 15, 1);
}

__device__ __forceinline__ Ctr4 noise_block(uint32_t block, int tg, uint32_t trial, uint32_t stream,
                                            uint32_t k0, uint32_t k1) {
  return philox4x32_10(Ctr4{block, (uint32_t)tg, trial, (kDomainNoise << 24) | stream}, k0, k1);
}

// I' = Q . S for row tile mt (before scale and h).
template <int NT, int PREC>
__device__ __forceinline__ void real_row_tile(const unsigned char* sJ, int lane, int mt,
                                              const v4i (&B)[NT][words<PREC>()], v16f& acc) {
  acc = v16f{};
  if constexpr (PREC == PIM_PREC_FP8) {
    constexpr int NK = (NT + 1) / 2;
    const v8i* f = reinterpret_cast<const v8i*>(sJ) + lane;
#pragma unroll
    for (int kk = 0; kk < NK; ++kk) {
      const v8i A = f[(mt * NK + kk) * 64];
      const v4i b0 = B[2 * kk][0];
      const v4i b1 = (2 * kk + 1 < NT) ? B[2 * kk + 1 < NT ? 2 * kk + 1 : 0][0] : v4i{0, 0, 0, 0};
      const v8i Bv = __builtin_shufflevector(b0, b1, 0, 1, 2, 3, 4, 5, 6, 7);
      acc = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(A, Bv, acc, 0, 0, 0, 0, 0, 0);
    }
  } else {
    const v4i* f = reinterpret_cast<const v4i*>(sJ) + lane;
#pragma unroll
    for (int kt = 0; kt < NT; ++kt)
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        const v4i A = f[((mt * NT + kt) * 2 + j) * 64];
        acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(v8bf, A), __builtin_bit_cast(v8bf, B[kt][j]),
                                                      acc, 0, 0, 0);
      }
  }
}

// Field thresholds of one row tile's 16 spins of a lane: tab[u ^ m] with u the
// noise byte and m the spin's sign mask.
template <int PREC>
__device__ __forceinline__ void real_tile_thresholds(const float* tab, const uint32_t (&xw)[4],
                                                     const uint32_t (&sw)[4 * words<PREC>()], float (&th)[16],
                                                     int (&sm)[16]) {
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    sm[r] = spin_mask<PREC>(sw, r);
    const int idx = (int)((xw[r >> 2] >> (8 * (r & 3))) & 0xFFu) ^ sm[r];
    th[r] = tab[idx];
  }
}

// v of the lane plus v of the lane 32 away (the two halves of a trial
// column): the lower half's value first, so every lane gets the same sum.
// One VALU lane swap instead of an LDS round trip.
__device__ __forceinline__ float half_sum(float v) {
  const auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(v), __float_as_uint(v), false, false);
  return __uint_as_float(r[0]) + __uint_as_float(r[1]);
}

// Decisions (Eq. (4)) and energy terms (Eq. (1)) of one row tile's 16 spins
// of a lane: I = scale * acc + h, new spins into bn (operand encoding), and
// the tile's energy sum pt = sum_r s_r (I_r + h_r), added from zero in r order.
template <int PREC, bool HAS_H>
__device__ __forceinline__ float real_tile_apply(const v16f& acc, float scale, const float* sH, int hoff,
                                                 const float (&th)[16], const int (&sm)[16],
                                                 v4i (&bn)[words<PREC>()]) {
  float pt = 0.0f;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    float d[4];
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      const int r = 4 * q + b;
      float I, v;
      if (HAS_H) {
        const float hv = sH[hoff + r];
        I = fmaf(scale, acc[r], hv);
        v = I + hv;
      } else {
        I = scale * acc[r];
        v = I;
      }
      pt += __uint_as_float(__float_as_uint(v) ^ ((uint32_t)sm[r] & 0x80000000u));  // s * v
      d[b] = I - th[r];  // sign bit set <=> s(t+1) = -1
    }
    const uint32_t d0 = __float_as_uint(d[0]), d1 = __float_as_uint(d[1]);
    const uint32_t d2 = __float_as_uint(d[2]), d3 = __float_as_uint(d[3]);
    if (PREC == PIM_PREC_FP8) {
      const uint32_t sgn = perm(d1, d0, 0x0C0C0B09u) | perm(d3, d2, 0x0B090C0Cu);
      bn[0][q] = (int)((sgn & 0x80808080u) | 0x38383838u);
    } else {
      bn[q >> 1][2 * (q & 1)] = (int)((perm(d1, d0, 0x0B0C090Cu) & 0x80008000u) | 0x3F803F80u);
      bn[q >> 1][2 * (q & 1) + 1] = (int)((perm(d3, d2, 0x0B0C090Cu) & 0x80008000u) | 0x3F803F80u);
    }
  }
  return pt;
}

// int8 spin bytes of one row tile's 16 spins of a lane from operand words
template <int PREC>
__device__ __forceinline__ v4i real_tile_i8(const v4i (&w)[words<PREC>()]) {
  v4i o;
  if (PREC == PIM_PREC_FP8) {
    for (int q = 0; q < 4; ++q) o[q] = (int)i8_from_fp8((uint32_t)w[0][q]);
  } else {
    for (int q = 0; q < 4; ++q) o[q] = (int)i8_from_bf16((uint32_t)w[q >> 1][2 * (q & 1)], (uint32_t)w[q >> 1][2 * (q & 1) + 1]);
  }
  return o;
}

template <int NT, int PREC, bool HAS_H>
__global__ __launch_bounds__(64 * kMaxWaves) void sweep_real_kernel(SweepRealArgs a) {
  extern __shared__ __align__(16) unsigned char lds[];
  constexpr int KW = words<PREC>();
  constexpr int kFragBytes = (int)frag_bytes(PREC, NT);
  constexpr int kNpad = NT * 32;
  constexpr int kHBytes = HAS_H ? kNpad * 4 : 0;
  const int nw = blockDim.x >> 6;
  const int inst = blockIdx.y;
  const int wave = threadIdx.x >> 6;
  const int lane = threadIdx.x & 63;
  const int col = lane & 31;
  const int half = lane >> 5;

  {  // stage the instance: quantised couplings and h
    const uint4* src = reinterpret_cast<const uint4*>(a.jfrag + (size_t)inst * kFragBytes);
    uint4* dst = reinterpret_cast<uint4*>(lds);
    for (int i = threadIdx.x; i < kFragBytes / 16; i += blockDim.x) dst[i] = src[i];
    if (HAS_H) {
      float* sh = reinterpret_cast<float*>(lds + kFragBytes);
      for (int i = threadIdx.x; i < kNpad; i += blockDim.x) sh[i] = a.h[(size_t)inst * kNpad + i];
    }
  }
  const unsigned char* sJ = lds;
  const float* sH = reinterpret_cast<const float*>(lds + kFragBytes);
  float* sTab = reinterpret_cast<float*>(lds + kFragBytes + kHBytes + wave * kRealTabBytes);
  uint4* sTab4 = reinterpret_cast<uint4*>(sTab);
  __syncthreads();  // the only workgroup barrier

  const int tbase = (blockIdx.x * nw + wave) * 32;
  if (tbase >= a.R) return;
  const int trial = tbase + col;
  const bool live = trial < a.R;
  const size_t cell = (size_t)inst * a.R + trial;
  const uint32_t stream = a.inst_stream[inst];
  const int cls = a.inst_class[inst];
  const uint4* gTab4 = reinterpret_cast<const uint4*>(a.thtab + (size_t)cls * a.T * kTabEntries);
  const float target = a.target ? a.target[inst] : -INFINITY;
  const float scale = a.scale[inst];
  const uint32_t k0 = a.k0, k1 = a.k1;

  // ---- s(0) ----
  v4i B[NT][KW];
#pragma unroll
  for (int mt = 0; mt < NT; ++mt) {
    uint32_t w[4];
    if (a.init) {
      const v4i v = live ? *reinterpret_cast<const v4i*>(a.init + cell * kNpad + 32 * mt + 16 * half)
                         : v4i{0x01010101, 0x01010101, 0x01010101, 0x01010101};
      for (int q = 0; q < 4; ++q) w[q] = (uint32_t)v[q];
    } else {
      const Ctr4 x = philox4x32_10(Ctr4{(uint32_t)(2 * mt + half), 0u, (uint32_t)trial,
                                        (kDomainInit << 24) | stream}, k0, k1);
      w[0] = spins_from_bits(x.x);
      w[1] = spins_from_bits(x.y);
      w[2] = spins_from_bits(x.z);
      w[3] = spins_from_bits(x.w);
    }
    if (PREC == PIM_PREC_FP8) {
      for (int q = 0; q < 4; ++q) B[mt][0][q] = (int)fp8_from_i8(w[q]);
    } else {
      for (int q = 0; q < 4; ++q) {
        B[mt][q >> 1][2 * (q & 1)] = (int)bf16_lo_from_i8(w[q]);
        B[mt][q >> 1][2 * (q & 1) + 1] = (int)bf16_hi_from_i8(w[q]);
      }
    }
  }

  float e_best = INFINITY, e_cur = 0.0f;
  int32_t t_best = -1, first_hit = -1;
  Ctr4 x_next = noise_block((uint32_t)half, a.start_step, (uint32_t)trial, stream, k0, k1);
  int done = a.T;
  sTab4[lane] = gTab4[lane];
  sTab4[64 + lane] = gTab4[64 + lane];
  // ring[i] holds the table of step t + 1 + i (clamped index: in bounds)
  uint4 ring[kAhead][2];
#pragma unroll
  for (int i = 0; i < kAhead; ++i) {
    const size_t row = (size_t)min(1 + i, a.T - 1) * 128;
    ring[i][0] = gTab4[row + lane];
    ring[i][1] = gTab4[row + 64 + lane];
  }

  for (int t = 0;; ++t) {
    const int tg = a.start_step + t;
    float ep = 0.0f;
    v4i Bn[NT][KW];
    const bool last = (t == a.T);
    const bool has_next = t + 1 < a.T;
    const uint4 nxt0 = ring[0][0];
    const uint4 nxt1 = ring[0][1];
#pragma unroll
    for (int i = 0; i + 1 < kAhead; ++i) {
      ring[i][0] = ring[i + 1][0];
      ring[i][1] = ring[i + 1][1];
    }
    {
      const size_t row = (size_t)min(t + 1 + kAhead, a.T - 1) * 128;
      ring[kAhead - 1][0] = gTab4[row + lane];
      ring[kAhead - 1][1] = gTab4[row + 64 + lane];
    }
    const float* tab = sTab + kNoiseVals;
    uint32_t ctr_trial = (uint32_t)trial;
    uint32_t ctr_half = (uint32_t)half;
    PIM_FENCE(ctr_trial);
    PIM_FENCE(ctr_half);
    v16f acc_next;
    real_row_tile<NT, PREC>(sJ, lane, 0, B, acc_next);
#pragma unroll
    for (int mt = 0; mt < NT; ++mt) {
      const v16f acc = acc_next;
      uint32_t xw[4] = {x_next.x, x_next.y, x_next.z, x_next.w};
      uint32_t sw[4 * KW];
#pragma unroll
      for (int q = 0; q < 4; ++q) PIM_FENCE(xw[q]);
#pragma unroll
      for (int q = 0; q < 4 * KW; ++q) {
        sw[q] = (uint32_t)B[mt][q >> 2][q & 3];
        PIM_FENCE(sw[q]);
      }
      int lane_off = lane;
      PIM_FENCE(lane_off);
      int hoff = 32 * mt + 16 * half;
      if (HAS_H) PIM_FENCE(hoff);
      // (1) LDS: the field thresholds of this tile
      float th[16];
      int sm[16];
      real_tile_thresholds<PREC>(tab, xw, sw, th, sm);
      // (2) the next tile's MFMA chain and noise block
      if (mt + 1 < NT) real_row_tile<NT, PREC>(sJ, lane_off, mt + 1, B, acc_next);
      if (mt + 1 < NT) x_next = noise_block(2u * (mt + 1) + ctr_half, tg, ctr_trial, stream, k0, k1);
      else x_next = noise_block(ctr_half, tg + 1, ctr_trial, stream, k0, k1);
      // (3) energy of s(t) and the decisions of this tile; tile sums are
      //     added in tile order (the order the split kernel reproduces)
      ep += real_tile_apply<PREC, HAS_H>(acc, scale, sH, hoff, th, sm, Bn[mt]);
      PIM_FENCE(ep);
#pragma unroll
      for (int j = 0; j < KW; ++j)
#pragma unroll
        for (int q = 0; q < 4; ++q) PIM_FENCE(Bn[mt][j][q]);
      __builtin_amdgcn_sched_barrier(0);
    }
    const float E = -0.5f * half_sum(ep);
    if (E < e_best) {
      e_best = E;
      t_best = tg;
      if (live) {
        size_t off = cell * kNpad + 16 * half;
        PIM_FENCE(off);
        int8_t* dst = a.best_s + off;
#pragma unroll
        for (int mt = 0; mt < NT; ++mt) *reinterpret_cast<v4i*>(dst + 32 * mt) = real_tile_i8<PREC>(B[mt]);
      }
    }
    if (first_hit < 0 && E <= target) first_hit = tg;
    e_cur = E;
    if (last) break;
    if ((t & 255) == 0 && __atomic_load_n(a.cancel, __ATOMIC_RELAXED) != 0) {
      done = t;
      break;
    }
#pragma unroll
    for (int mt = 0; mt < NT; ++mt)
#pragma unroll
      for (int j = 0; j < KW; ++j) B[mt][j] = Bn[mt][j];
    if (has_next) {
      sTab4[lane] = nxt0;
      sTab4[64 + lane] = nxt1;
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
  }

  if (!live) return;
#pragma unroll
  for (int mt = 0; mt < NT; ++mt)
    *reinterpret_cast<v4i*>(a.final_s + cell * kNpad + 32 * mt + 16 * half) = real_tile_i8<PREC>(B[mt]);
  if (half == 0) {
    a.e_best[cell] = e_best;
    a.t_best[cell] = t_best;
    a.first_hit[cell] = first_hit;
    a.e_final[cell] = e_cur;
    a.steps_done[cell] = done;
  }
}

// Latency form of the sweep for launches with few 32-trial blocks (a single
// request, a small chunk): W waves share one 32-trial block and split its row
// tiles (wave w owns mt = w, w + W, ...), so a step's decisions run on W SIMDs
// at once instead of one after another.  The spins of s(t) are exchanged
// through a double-buffered LDS copy of the B-operand words (each wave writes
// the words of its own tiles for s(t+1)); the step table is shared and
// double-buffered; the tile energy sums go to LDS and every lane adds them in
// tile order after the step's single barrier, which gives exactly the
// one-wave kernel's energies.  A buffer is rewritten two steps after it was
// read, and every wave has passed the barrier in between.
template <int NT, int PREC, bool HAS_H, int W>
__global__ __launch_bounds__(64 * W) void sweep_real_split_kernel(SweepRealArgs a) {
  extern __shared__ __align__(16) unsigned char lds[];
  constexpr int KW = words<PREC>();
  constexpr int kFragBytes = (int)frag_bytes(PREC, NT);
  constexpr int kNpad = NT * 32;
  constexpr int kHBytes = HAS_H ? kNpad * 4 : 0;
  constexpr int RPW = (NT + W - 1) / W;
  // LDS: fragments | h | spin words [2][NT][KW][64] v4i | tables [2][kTabEntries]
  // | tile energy sums [2][NT][64] | cancel flag
  v4i* sS = reinterpret_cast<v4i*>(lds + kFragBytes + kHBytes);
  float* sTab = reinterpret_cast<float*>(sS + 2 * NT * KW * 64);
  float* sP = sTab + 2 * kTabEntries;
  int32_t* sFlag = reinterpret_cast<int32_t*>(sP + 2 * NT * 64);
  const int inst = blockIdx.y;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  const int col = lane & 31;
  const int half = lane >> 5;
  {  // stage the instance: quantised couplings and h
    const uint4* src = reinterpret_cast<const uint4*>(a.jfrag + (size_t)inst * kFragBytes);
    uint4* dst = reinterpret_cast<uint4*>(lds);
    for (int i = threadIdx.x; i < kFragBytes / 16; i += blockDim.x) dst[i] = src[i];
    if (HAS_H) {
      float* sh = reinterpret_cast<float*>(lds + kFragBytes);
      for (int i = threadIdx.x; i < kNpad; i += blockDim.x) sh[i] = a.h[(size_t)inst * kNpad + i];
    }
  }
  const unsigned char* sJ = lds;
  const float* sH = reinterpret_cast<const float*>(lds + kFragBytes);
  const int trial = blockIdx.x * 32 + col;
  const bool live = trial < a.R;
  const size_t cell = (size_t)inst * a.R + trial;
  const uint32_t stream = a.inst_stream[inst];
  const int cls = a.inst_class[inst];
  const uint4* gTab4 = reinterpret_cast<const uint4*>(a.thtab + (size_t)cls * a.T * kTabEntries);
  const float target = a.target ? a.target[inst] : -INFINITY;
  const float scale = a.scale[inst];
  const uint32_t k0 = a.k0, k1 = a.k1;
  auto word = [&](int buf, int mt, int j) -> v4i& { return sS[((buf * NT + mt) * KW + j) * 64 + lane]; };

  // ---- s(0): each wave its own row tiles ----
#pragma unroll
  for (int jj = 0; jj < RPW; ++jj) {
    const int mt = wave + W * jj;
    if (mt >= NT) break;  // uniform
    uint32_t w[4];
    if (a.init) {
      const v4i v = live ? *reinterpret_cast<const v4i*>(a.init + cell * kNpad + 32 * mt + 16 * half)
                         : v4i{0x01010101, 0x01010101, 0x01010101, 0x01010101};
      for (int q = 0; q < 4; ++q) w[q] = (uint32_t)v[q];
    } else {
      const Ctr4 x = philox4x32_10(Ctr4{(uint32_t)(2 * mt + half), 0u, (uint32_t)trial,
                                        (kDomainInit << 24) | stream}, k0, k1);
      w[0] = spins_from_bits(x.x);
      w[1] = spins_from_bits(x.y);
      w[2] = spins_from_bits(x.z);
      w[3] = spins_from_bits(x.w);
    }
    v4i b[KW];
    if (PREC == PIM_PREC_FP8) {
      for (int q = 0; q < 4; ++q) b[0][q] = (int)fp8_from_i8(w[q]);
    } else {
      for (int q = 0; q < 4; ++q) {
        b[q >> 1][2 * (q & 1)] = (int)bf16_lo_from_i8(w[q]);
        b[q >> 1][2 * (q & 1) + 1] = (int)bf16_hi_from_i8(w[q]);
      }
    }
#pragma unroll
    for (int j = 0; j < KW; ++j) word(0, mt, j) = b[j];
  }
  // the step tables move through LDS as kTabVec 16-byte words, spread over
  // every thread of the block (kTabPer words each; with more threads than
  // words the last word is loaded and stored by several threads, all with the
  // same value, so no access needs a branch)
  constexpr int kTabVec = kTabEntries / 4;
  constexpr int kTabPer = (kTabVec + 64 * W - 1) / (64 * W);
  uint4* sTab4 = reinterpret_cast<uint4*>(sTab);
  auto tab_word = [&](int i) { return min((int)threadIdx.x + 64 * W * i, kTabVec - 1); };
#pragma unroll
  for (int i = 0; i < kTabPer; ++i) sTab4[tab_word(i)] = gTab4[tab_word(i)];
  if (threadIdx.x == 0) sFlag[0] = 0;
  __syncthreads();

  float e_best = INFINITY, e_cur = 0.0f;
  int32_t t_best = -1, first_hit = -1;
  int done = a.T;
  // The next tables are held in registers, in two sets used by alternate
  // steps: a table is loaded two steps before it is stored to LDS (three
  // before it is used), in place, because one step is shorter than the load's
  // latency from a cache of another chiplet; no register copy waits on a
  // load (clamped index: in bounds).  The best state stays in registers and
  // is stored once after the step loop, so the loop issues no global store
  // and the table loads are the only memory operations a wait counts.
  uint4 trA[kTabPer], trB[kTabPer];
#pragma unroll
  for (int i = 0; i < kTabPer; ++i) {
    trA[i] = gTab4[(size_t)min(1, a.T - 1) * kTabVec + tab_word(i)];
    trB[i] = gTab4[(size_t)min(2, a.T - 1) * kTabVec + tab_word(i)];
  }
  v4i Bb[RPW][KW];  // s(t) of the best energy so far, own tiles
  auto store_best = [&]() {
    size_t off = cell * kNpad + 16 * half;
    PIM_FENCE(off);
    int8_t* dst = a.best_s + off;
#pragma unroll
    for (int jj = 0; jj < RPW; ++jj) {
      const int mt = wave + W * jj;
      if (mt < NT) *reinterpret_cast<v4i*>(dst + 32 * mt) = real_tile_i8<PREC>(Bb[jj]);
    }
  };
  // the start of step t: the table of step t+1 into the other buffer (last
  // read in step t-1, before the barrier every thread has passed since), then
  // the load of the table of step t+3 into the same registers
  auto step_tables = [&](int t, uint4 (&tr)[kTabPer]) __attribute__((always_inline)) {
    const int nxt = (t & 1) ^ 1;
#pragma unroll
    for (int i = 0; i < kTabPer; ++i) sTab4[nxt * kTabVec + tab_word(i)] = tr[i];
    const size_t row = (size_t)min(t + 3, a.T - 1) * kTabVec;
#pragma unroll
    for (int i = 0; i < kTabPer; ++i) tr[i] = gTab4[row + tab_word(i)];
  };
  // the rest of step t; true when the run ends after it.  The loop below
  // alternates the register set, so each set is a constant in its copy of the
  // step, and runs the next step's tables at the end of each step, so the
  // loop header uses no loaded register.  t is even in the first copy, which
  // alone can meet the cancel poll (every 256 steps).
  auto step = [&](int t, auto even_c) __attribute__((always_inline)) -> bool {
    constexpr bool EVEN = decltype(even_c)::value;
    const int tg = a.start_step + t;
    const int cur = t & 1, nxt = cur ^ 1;
    uint32_t ctr_trial = (uint32_t)trial, ctr_half = (uint32_t)half;
    PIM_FENCE(ctr_trial);
    PIM_FENCE(ctr_half);
    v4i B[NT][KW];  // s(t), all tiles
#pragma unroll
    for (int mt = 0; mt < NT; ++mt)
#pragma unroll
      for (int j = 0; j < KW; ++j) B[mt][j] = word(cur, mt, j);
    // noise blocks of the wave's tiles, issued after the spin-word reads:
    // independent of the spins, they cover that latency and the MFMAs'
    Ctr4 xs[RPW];
#pragma unroll
    for (int jj = 0; jj < RPW; ++jj) {
      const int mt = wave + W * jj;
      if (mt < NT) xs[jj] = noise_block(2u * mt + ctr_half, tg, ctr_trial, stream, k0, k1);
    }
    const float* tab = sTab + cur * kTabEntries + kNoiseVals;
#pragma unroll
    for (int jj = 0; jj < RPW; ++jj) {
      const int mt = wave + W * jj;
      if (mt >= NT) break;  // uniform
      v16f acc;
      real_row_tile<NT, PREC>(sJ, lane, mt, B, acc);
      uint32_t xw[4] = {xs[jj].x, xs[jj].y, xs[jj].z, xs[jj].w};
      uint32_t sw[4 * KW];
#pragma unroll
      for (int q = 0; q < 4 * KW; ++q) sw[q] = (uint32_t)B[mt][q >> 2][q & 3];
      float th[16];
      int sm[16];
      real_tile_thresholds<PREC>(tab, xw, sw, th, sm);
      v4i bn[KW];
      const float pt = real_tile_apply<PREC, HAS_H>(acc, scale, sH, 32 * mt + 16 * half, th, sm, bn);
      sP[(cur * NT + mt) * 64 + lane] = pt;
#pragma unroll
      for (int j = 0; j < KW; ++j) word(nxt, mt, j) = bn[j];
      __builtin_amdgcn_sched_barrier(0);
    }
    if (EVEN && threadIdx.x == 0 && (t & 255) == 0 && t < a.T)
      sFlag[0] = __atomic_load_n(a.cancel, __ATOMIC_RELAXED) != 0 ? 1 : 0;
    lds_barrier();  // s(t+1), the tile energy sums of s(t) and the next table are complete
    float ep = 0.0f;
#pragma unroll
    for (int mt = 0; mt < NT; ++mt) ep += sP[(cur * NT + mt) * 64 + lane];  // tile order
    const float E = -0.5f * half_sum(ep);
    if (E < e_best) {
      e_best = E;
      t_best = tg;
      if (live) {
#pragma unroll
        for (int jj = 0; jj < RPW; ++jj) {
          const int mt = wave + W * jj;
          if (mt < NT)
#pragma unroll
            for (int j = 0; j < KW; ++j) Bb[jj][j] = B[mt][j];
        }
      }
    }
    if (first_hit < 0 && E <= target) first_hit = tg;
    e_cur = E;
    if (t == a.T) return true;  // uniform: s(T) is in B
    const bool stop = EVEN && (t & 255) == 0 && sFlag[0] != 0;  // uniform: written before the barrier
    if (stop) {
      done = t;  // s(t) stays the final state
      return true;
    }
    return false;
  };
  step_tables(0, trA);
  for (int t = 0;; t += 2) {
    if (step(t, std::true_type{})) break;
    step_tables(t + 1, trB);
    if (step(t + 1, std::false_type{})) break;
    step_tables(t + 2, trA);
  }
  if (live && t_best >= 0) store_best();
  // the final state s(t) is in B (every wave holds all tiles; each writes its own)
  if (!live) return;
  {
    v4i B[NT][KW];
    const int last = (done == a.T ? a.T : done) & 1;
#pragma unroll
    for (int mt = 0; mt < NT; ++mt)
#pragma unroll
      for (int j = 0; j < KW; ++j) B[mt][j] = word(last, mt, j);
#pragma unroll
    for (int jj = 0; jj < RPW; ++jj) {
      const int mt = wave + W * jj;
      if (mt < NT) *reinterpret_cast<v4i*>(a.final_s + cell * kNpad + 32 * mt + 16 * half) = real_tile_i8<PREC>(B[mt]);
    }
  }
  if (wave == 0 && half == 0) {
    a.e_best[cell] = e_best;
    a.t_best[cell] = t_best;
    a.first_hit[cell] = first_hit;
    a.e_final[cell] = e_cur;
    a.steps_done[cell] = done;
  }
}

constexpr int kSplitMaxBlocks = 128;  // 32-trial blocks per launch up to which the split form runs

template <int NT, int PREC, bool HAS_H>
constexpr size_t split_lds_bytes() {
  return frag_bytes(PREC, NT) + (HAS_H ? NT * 32 * 4 : 0) + (size_t)2 * NT * words<PREC>() * 1024 +
         (size_t)2 * kTabEntries * 4 + (size_t)2 * NT * 64 * 4 + 16;
}

template <int NT, int PREC, bool HAS_H>
hipError_t launch_split(const SweepRealArgs& a, int count, hipStream_t s) {
  // one row tile per wave up to 4 tiles; above, eight waves (two per SIMD):
  // at N = 256 a request took 90 us against 115 us with four waves of two
  // tiles each
  constexpr int W = NT <= 4 ? NT : 8;
  constexpr size_t lds = split_lds_bytes<NT, PREC, HAS_H>();
  auto kern = sweep_real_split_kernel<NT, PREC, HAS_H, W>;
  hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  const dim3 grid((a.R + 31) / 32, count);
  hipLaunchKernelGGL(kern, grid, dim3(64 * W), lds, s, a);
  return hipGetLastError();
}

template <int NT, int PREC, bool HAS_H>
hipError_t launch_nt(const SweepRealArgs& a, int count, hipStream_t s) {
  // few trial blocks: the latency form (when its LDS fits)
  if (NT > 1 && (size_t)count * ((a.R + 31) / 32) <= (size_t)kSplitMaxBlocks &&
      split_lds_bytes<NT, PREC, HAS_H>() <= (size_t)160 * 1024)
    return launch_split<NT, PREC, HAS_H>(a, count, s);
  const int nw = std::min(kMaxWaves, (a.R + 31) / 32);
  const size_t lds = frag_bytes(PREC, NT) + (HAS_H ? NT * 32 * 4 : 0) + (size_t)nw * kRealTabBytes;
  auto kern = sweep_real_kernel<NT, PREC, HAS_H>;
  hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  const dim3 grid((a.R + 32 * nw - 1) / (32 * nw), count);
  hipLaunchKernelGGL(kern, grid, dim3(64 * nw), lds, s, a);
  return hipGetLastError();
}

template <int PREC, bool HAS_H>
hipError_t launch_p(const SweepRealArgs& a, int count, int nt, hipStream_t s) {
  switch (nt) {
    case 1: return launch_nt<1, PREC, HAS_H>(a, count, s);
    case 2: return launch_nt<2, PREC, HAS_H>(a, count, s);
    case 3: return launch_nt<3, PREC, HAS_H>(a, count, s);
    case 4: return launch_nt<4, PREC, HAS_H>(a, count, s);
    case 5: return launch_nt<5, PREC, HAS_H>(a, count, s);
    case 6: return launch_nt<6, PREC, HAS_H>(a, count, s);
    case 7: return launch_nt<7, PREC, HAS_H>(a, count, s);
    case 8: return launch_nt<8, PREC, HAS_H>(a, count, s);
    default: return hipErrorInvalidValue;
  }
}

// Device quantisers: the same round-to-nearest-even from binary64 as the host
// ones (frexp, ldexp and rint are exact), so both produce identical codes.
__device__ uint8_t d_fp8(double x) {
  if (x == 0.0 || isnan(x)) return 0;
  const uint8_t sign = x < 0.0 ? 0x80 : 0x00;
  const double a = fabs(x);
  if (a >= 448.0) return sign | 0x7E;
  if (a < 0.015625) return sign | (uint8_t)rint(a * 512.0);
  int e;
  (void)frexp(a, &e);
  int E = e - 1;
  double q = rint(ldexp(a, 3 - E));
  if (q == 16.0) {
    q = 8.0;
    ++E;
  }
  if (E > 8 || (E == 8 && q > 14.0)) return sign | 0x7E;
  return sign | (uint8_t)(((E + 7) << 3) | ((int)q - 8));
}

__device__ uint16_t d_bf16(double x) {
  if (x == 0.0 || isnan(x)) return 0;
  const uint16_t sign = x < 0.0 ? 0x8000 : 0x0000;
  if (isinf(x)) return sign | 0x7F80;
  const double a = fabs(x);
  int e;
  (void)frexp(a, &e);
  int E = e - 1;
  if (E < -126) return sign | (uint16_t)rint(ldexp(a, 133));
  double q = rint(ldexp(a, 7 - E));
  if (q == 256.0) {
    q = 128.0;
    ++E;
  }
  if (E > 127) return sign | 0x7F80;
  return sign | (uint16_t)(((E + 127) << 7) | ((int)q - 128));
}

// Blocks (slice, inst): max |J| over one of kPackSlices equal slices of the
// instance's binary64 J (npad^2 is a multiple of kPackSlices).
__global__ __launch_bounds__(256) void max_slices_kernel(RealPackArgs a) {
  __shared__ double red[256];
  const int inst = blockIdx.y, np = a.npad;
  const int per = np * np / kPackSlices;
  const double* J = a.j64 + (size_t)inst * np * np + (size_t)blockIdx.x * per;
  double m = 0.0;
  for (int i = threadIdx.x; i < per; i += 256) m = fmax(m, fabs(J[i]));
  red[threadIdx.x] = m;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + w]);
    __syncthreads();
  }
  if (threadIdx.x == 0) a.pmax[(size_t)inst * kPackSlices + blockIdx.x] = red[0];
}

// Blocks (x, inst): scale = max|J| / 448 (FP8, rounded to binary32) or the
// power of two with max|J| / scale in [1, 2) (BF16), formed by every block of
// the instance alike from the slice maxima; J / scale quantised into the
// fragment order of pack_real_fragments, each block taking every
// gridDim.x-th group of 256 outputs; h converted to binary32.  J and h are
// the instance's binary64 values, zero-padded to npad.
template <int PREC>
__global__ __launch_bounds__(256) void pack_real_kernel(RealPackArgs a) {
  const int inst = blockIdx.y;
  const int first = blockIdx.x * 256 + threadIdx.x, step = gridDim.x * 256;
  const int np = a.npad, nt = np / 32;
  const double* J = a.j64 + (size_t)inst * np * np;
  double m = 0.0;
  for (int q = 0; q < kPackSlices; ++q) m = fmax(m, a.pmax[(size_t)inst * kPackSlices + q]);
  float scale = 1.0f;
  if (m > 0.0) {
    if (PREC == PIM_PREC_FP8) {
      scale = (float)(m / 448.0);
    } else {
      int e;
      (void)frexp(m, &e);
      scale = (float)ldexp(1.0, e - 1);
    }
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) a.scale[inst] = scale;
  auto row_of = [](int mt, int r) { return 32 * mt + 16 * ((r >> 2) & 1) + 4 * (r >> 3) + (r & 3); };
  uint8_t* out = a.frag + (size_t)inst * a.frag_bytes;
  if (PREC == PIM_PREC_FP8) {
    const int nk = (nt + 1) / 2;
    const int total = nt * nk * 64 * 32;
    for (int b = first; b < total; b += step) {
      const int p = b & 31, l = (b >> 5) & 63, blk = b >> 11;  // blk = mt * nk + kk
      const int mt = blk / nk, kk = blk % nk;
      const int row = row_of(mt, l & 31);
      const int colj = 32 * (2 * kk + p / 16) + 16 * (l >> 5) + (p % 16);
      const double v = (colj < np) ? J[(size_t)row * np + colj] / (double)scale : 0.0;
      out[b] = d_fp8(v);
    }
  } else {
    uint16_t* o16 = reinterpret_cast<uint16_t*>(out);
    const int total = nt * nt * 2 * 64 * 8;
    for (int b = first; b < total; b += step) {
      const int p = b & 7, l = (b >> 3) & 63, blk = b >> 9;  // blk = (mt * nt + kt) * 2 + j
      const int j = blk & 1, kt = (blk >> 1) % nt, mt = (blk >> 1) / nt;
      const int row = row_of(mt, l & 31);
      const int colj = 32 * kt + 16 * (l >> 5) + 8 * j + p;
      o16[b] = d_bf16(J[(size_t)row * np + colj] / (double)scale);
    }
  }
  for (int i = first; i < np; i += step) a.hf[(size_t)inst * np + i] = (float)a.h64[(size_t)inst * np + i];
}

}  // namespace

size_t real_frag_bytes(int prec, int nt) { return frag_bytes(prec, nt); }

hipError_t launch_pack_real(const RealPackArgs& a, int prec, hipStream_t s) {
  if (a.count < 1) return hipSuccess;
  if (a.npad < 32 || a.npad > PIM_MAX_N_LDS || a.npad % 32) return hipErrorInvalidValue;
  hipLaunchKernelGGL(max_slices_kernel, dim3(kPackSlices, a.count), dim3(256), 0, s, a);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  // blocks per instance: one per 4096 coupling elements (1 at N = 32, 16 at N = 256)
  const dim3 grid(std::max(1, a.npad * a.npad / 4096), a.count);
  if (prec == PIM_PREC_FP8) hipLaunchKernelGGL(pack_real_kernel<PIM_PREC_FP8>, grid, dim3(256), 0, s, a);
  else if (prec == PIM_PREC_BF16) hipLaunchKernelGGL(pack_real_kernel<PIM_PREC_BF16>, grid, dim3(256), 0, s, a);
  else return hipErrorInvalidValue;
  return hipGetLastError();
}

hipError_t launch_sweep_real(const SweepRealArgs& a, int count, int nt, int prec, bool has_h, hipStream_t s) {
  if (a.npad != nt * 32 || a.R < 1) return hipErrorInvalidValue;
  if (prec == PIM_PREC_FP8)
    return has_h ? launch_p<PIM_PREC_FP8, true>(a, count, nt, s) : launch_p<PIM_PREC_FP8, false>(a, count, nt, s);
  if (prec == PIM_PREC_BF16)
    return has_h ? launch_p<PIM_PREC_BF16, true>(a, count, nt, s) : launch_p<PIM_PREC_BF16, false>(a, count, nt, s);
  return hipErrorInvalidValue;
}

void pack_real_fragments(const double* J, int n, int nt, int prec, float scale, uint8_t* out) {
  auto row_of = [](int mt, int m) { return 32 * mt + 16 * ((m >> 2) & 1) + 4 * (m >> 3) + (m & 3); };
  if (prec == PIM_PREC_FP8) {
    const int nk = (nt + 1) / 2;
    for (int mt = 0; mt < nt; ++mt)
      for (int kk = 0; kk < nk; ++kk)
        for (int l = 0; l < 64; ++l) {
          const int row = row_of(mt, l & 31), hh = l >> 5;
          for (int p = 0; p < 32; ++p) {
            const int colj = 32 * (2 * kk + p / 16) + 16 * hh + (p % 16);
            const double v = (row < n && colj < n) ? J[(size_t)row * n + colj] / (double)scale : 0.0;
            out[(((size_t)mt * nk + kk) * 64 + l) * 32 + p] = fp8_e4m3_rne(v);
          }
        }
  } else {
    uint16_t* o16 = reinterpret_cast<uint16_t*>(out);
    for (int mt = 0; mt < nt; ++mt)
      for (int kt = 0; kt < nt; ++kt)
        for (int j = 0; j < 2; ++j)
          for (int l = 0; l < 64; ++l) {
            const int row = row_of(mt, l & 31), hh = l >> 5;
            for (int p = 0; p < 8; ++p) {
              const int colj = 32 * kt + 16 * hh + 8 * j + p;
              const double v = (row < n && colj < n) ? J[(size_t)row * n + colj] / (double)scale : 0.0;
              o16[((((size_t)mt * nt + kt) * 2 + j) * 64 + l) * 8 + p] = bf16_rne(v);
            }
          }
  }
}

}  // namespace pim
