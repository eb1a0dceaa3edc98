// Persistent PIMI sweep with the couplings in LDS (N <= 256) on e2m1 (FP4)
// matrix cores, for integer instances whose couplings all lie in {0, +-1,
// +-2, +-3, +-4, +-6} (exact in e2m1).  It is the int8 LDS kernel's design --
// one workgroup per instance, each wave owning 32 trials and every spin row, a
// whole step inside the wave with no barrier -- with two changes:
//
//   * the contraction I[Npad x 32] = J'[Npad x Npad] . S[Npad x 32] runs on
//     v_mfma_f32_32x32x64_f8f6f4 with both operands e2m1: ceil(NT / 2) MFMAs
//     per row tile instead of NT, and half the LDS bytes of J per tile;
//   * the spins enter as e2m1 +-2.0 (0x4 / 0xC), 4 bits each: the K step p
//     B operand is the lane's own nibble words of tiles 2p and 2p + 1, so the
//     C -> B hand-off still never leaves the lane, and the signed 2-bit field
//     at the top of a nibble is s itself.
//
// Every product is an exact integer and |2 I| <= 2 * 32766 < 2^17 (the row
// bound instances are validated against).  Each row tile's accumulation
// starts from 1.5 * 2^23 instead of 0, so every partial sum lies in
// [2^23, 2^24), where binary32 steps by exactly 1: the accumulator holds
// 1.5 * 2^23 + 2 I exactly in any accumulation order, and its bit pattern is
// the integer 0x4B400000 + 2 I.  The kernel compares that pattern with
// thresholds biased the same way (no float-to-int conversion), and
// accumulates the energy from its low 24 bits, 2^22 + 2 I (+ 4 h), removing
// the 2^22 s terms afterwards from a count of the negative spins.
// Trajectories, energies and best states are identical to the int8 kernel's.
//
// Spin layout as in the int8 kernel: register r of half hh of row tile mt is
// spin 32 mt + 16 hh + r.  As e2m1 a tile's 16 spins of a lane sit in two
// words q: byte b of word q holds spin 8q + b in its low nibble and spin
// 8q + 4 + b in its high nibble (the order pack_f4_fragments packs J's K
// dimension in).
#include <hip/hip_runtime.h>

#include <climits>
#include <cstdint>

#include "internal.hpp"
#include "philox.hpp"
#include "e2m1.hpp"

namespace pim {
namespace {

using namespace e2m1;

constexpr int kWaves = 4;                      // most waves (32-trial blocks) per workgroup
constexpr int kXcds = 8;                  // XCDs of the device (workgroup placement)
constexpr float kAccBias = 12582912.0f;        // 1.5 * 2^23: start of every row tile's sum
constexpr int32_t kAccBiasBits = 0x4B400000;   // its bit pattern; + 2 I is the biased field
constexpr int32_t kLow24Bias = 0x400000;       // its low 24 bits: 2^22

#define PIM_FENCE(v) asm volatile("" : "+v"(v))

__device__ __forceinline__ Ctr4 noise_block(uint32_t block, int tg, uint32_t trial, uint32_t stream,
                                            uint32_t k0, uint32_t k1) {
  return philox4x32_10(Ctr4{block, (uint32_t)tg, trial, (kDomainNoise << 24) | stream}, k0, k1);
}

// K step p's B operand: the nibble words of tiles 2p and 2p + 1 (a tile past
// the last one has zero couplings; +2 stands in for its spins).
template <int NT>
__device__ __forceinline__ v4i b_operand(const uint2 (&S)[NT], int p) {
  const uint2 lo = S[2 * p];
  const uint2 hi = (2 * p + 1 < NT) ? S[2 * p + 1] : uint2{kPlusTwos, kPlusTwos};
  return v4i{(int)lo.x, (int)lo.y, (int)hi.x, (int)hi.y};
}

// 1.5 * 2^23 + 2 I for row tile mt: ceil(NT / 2) chained e2m1 MFMAs over the
// K steps, the first one adding to the bias registers.
template <int NT>
__device__ __forceinline__ v16f row_tile(const v4i* sJl, int mt, const uint2 (&S)[NT], const v16f& bias) {
  constexpr int NP = (NT + 1) / 2;
  v16f acc = mfma(sJl[(mt * NP) * 64], b_operand<NT>(S, 0), bias);
#pragma unroll
  for (int p = 1; p < NP; ++p) acc = mfma(sJl[(mt * NP + p) * 64], b_operand<NT>(S, p), acc);
  return acc;
}

// Step table into the wave's LDS buffer as biased doubled thresholds: lane l
// holds host entries 8l .. 8l + 7 (16-bit) and writes eight int32
// 0x4B400000 + 2 theta.
__device__ __forceinline__ void stage_table(int32_t* dst, uint4 v, int lane) {
  const uint32_t w[4] = {v.x, v.y, v.z, v.w};
  int32_t o[8];
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    o[2 * q] = ((int32_t)(w[q] << 16) >> 15) + kAccBiasBits;              // low half
    o[2 * q + 1] = ((int32_t)(w[q] & 0xFFFF0000u) >> 15) + kAccBiasBits;  // high half
  }
  reinterpret_cast<int4*>(dst)[2 * lane] = int4{o[0], o[1], o[2], o[3]};
  reinterpret_cast<int4*>(dst)[2 * lane + 1] = int4{o[4], o[5], o[6], o[7]};
}

// TAIL (4, 8, 12 or 16): registers of the last row tile that carry spins
// below N in the lower lane half, rounded up to 4; the others are padding
// spins (zero couplings) and keep their initial values.
template <int NT, bool HAS_H, int TAIL>
__global__ __launch_bounds__(64 * kWaves, 3) void sweep_mfma4_kernel(SweepArgs a, int blocks_per_inst) {
  extern __shared__ __align__(16) unsigned char lds[];
  constexpr int NP = (NT + 1) / 2;
  constexpr int kFragBytes = NT * NP * 1024;
  constexpr int kNpad = NT * 32;
  constexpr int kHBytes = HAS_H ? kNpad * 4 : 0;
  // workgroup -> (instance, trial block): the blocks of instance k have linear
  // ids congruent to k modulo the XCD count (consecutive workgroups go to
  // consecutive XCDs), so they run on one XCD and J is fetched into one L2
  const int lin = blockIdx.x;
  const int inst = (lin % kXcds) + kXcds * ((lin / kXcds) / blocks_per_inst);
  const int tblk = (lin / kXcds) % blocks_per_inst;
  if (inst >= a.count) return;  // whole workgroup, before any barrier
  const int wave = threadIdx.x >> 6;
  const int lane = threadIdx.x & 63;
  const int col = lane & 31;
  const int half = lane >> 5;

  {  // stage the instance: J fragments and 2 h
    const uint4* src = reinterpret_cast<const uint4*>(a.jfrag + (size_t)inst * kFragBytes);
    uint4* dst = reinterpret_cast<uint4*>(lds);
    for (int i = threadIdx.x; i < kFragBytes / 16; i += blockDim.x) dst[i] = src[i];
    if (HAS_H) {
      int32_t* sh = reinterpret_cast<int32_t*>(lds + kFragBytes);
      for (int i = threadIdx.x; i < kNpad; i += blockDim.x) sh[i] = 2 * a.h[(size_t)inst * kNpad + i];
    }
  }
  const v4i* sJ = reinterpret_cast<const v4i*>(lds);
  const int32_t* sH = reinterpret_cast<const int32_t*>(lds + kFragBytes);
  int32_t* sTab = reinterpret_cast<int32_t*>(lds + kFragBytes + kHBytes + wave * kTab32Bytes);
  __syncthreads();  // the only workgroup barrier

  const int trial = (tblk * (int)(blockDim.x >> 6) + wave) * 32 + col;
  if (trial - col >= a.R) return;  // whole wave
  const bool live = trial < a.R;
  const size_t cell = (size_t)inst * a.R + trial;
  const uint32_t stream = a.inst_stream[inst];
  const int cls = a.inst_class[inst];
  const uint4* gTab4 = reinterpret_cast<const uint4*>(a.thtab + (size_t)cls * a.T * kTabEntries);
  const int32_t target = a.target ? a.target[inst] : INT_MIN;
  const uint32_t k0 = a.k0, k1 = a.k1;

  // ---- s(0) ----
  uint2 S[NT];
#pragma unroll
  for (int mt = 0; mt < NT; ++mt) {
    v4i v;
    if (a.init) {
      v = live ? *reinterpret_cast<const v4i*>(a.init + cell * kNpad + 32 * mt + 16 * half)
               : v4i{0x01010101, 0x01010101, 0x01010101, 0x01010101};
    } else {
      const Ctr4 x = philox4x32_10(Ctr4{(uint32_t)(2 * mt + half), 0u, (uint32_t)trial,
                                        (kDomainInit << 24) | stream}, k0, k1);
      v = v4i{(int)spins_from_bits(x.x), (int)spins_from_bits(x.y), (int)spins_from_bits(x.z),
              (int)spins_from_bits(x.w)};
    }
    S[mt] = nib_tile(v);
  }

  int32_t e_best = INT_MAX, t_best = -1, first_hit = -1, e_cur = 0;
  Ctr4 x_next = noise_block((uint32_t)half, a.start_step, (uint32_t)trial, stream, k0, k1);
  int done = a.T;
  stage_table(sTab, gTab4[lane], lane);  // table of step 0
  // the accumulator start, kept in registers (fenced: not rematerialised as
  // sixteen moves before every row tile)
  v16f bias;
#pragma unroll
  for (int i = 0; i < 16; ++i) {
    float b = kAccBias;
    PIM_FENCE(b);
    bias[i] = b;
  }
  // the 2^22 s terms of one step's energy sums: 2^22 (decided spins - 2 negatives)
  constexpr int kDecided = 16 * (NT - 1) + TAIL;

  for (int t = 0;; ++t) {
    const int tg = a.start_step + t;
    // Same software pipeline as the int8 kernel: the MFMA chain of tile mt+1
    // and its noise block are issued before the decisions of tile mt.  At
    // t = T only the energy is used.
    int32_t ep = 0;
    uint2 Sn[NT];
    const bool last = (t == a.T);
    const bool has_next = t + 1 < a.T;
    const uint4 nxt = gTab4[(size_t)min(t + 1, a.T - 1) * 64 + lane];
    // centre of this step's table: entry u ^ s for s = +-1 (u ^ 1 / ~u)
    const int32_t* tab = sTab + kNoiseVals;
    uint32_t ctr_trial = (uint32_t)trial, ctr_half = (uint32_t)half;
    PIM_FENCE(ctr_half);
    PIM_FENCE(ctr_trial);
    const v4i* sJl0 = sJ + lane;
    v16f acc_next = row_tile<NT>(sJl0, 0, S, bias);
    int32_t nneg = 0;  // negative spins among this lane's decided registers
#pragma unroll
    for (int mt = 0; mt < NT; ++mt) {
      const v16f acc = acc_next;
      uint32_t xw[4] = {x_next.x, x_next.y, x_next.z, x_next.w};
      uint32_t sw[2] = {S[mt].x, S[mt].y};
#pragma unroll
      for (int q = 0; q < 4; ++q) PIM_FENCE(xw[q]);
      int lane_off = lane;
      PIM_FENCE(lane_off);
      int hoff = 32 * mt + 16 * half;
      if (HAS_H) PIM_FENCE(hoff);
      const v4i* sJl = sJ + lane_off;
      const int kRegs = (mt == NT - 1) ? TAIL : 16;
      // (1) LDS: the doubled thresholds of this tile, indexed by u ^ s
      int sv[16], th[16];
#pragma unroll
      for (int r = 0; r < kRegs; ++r) {
        sv[r] = spin_of(sw, r);
        th[r] = tab[(int)((xw[r >> 2] >> (8 * (r & 3))) & 0xFFu) ^ sv[r]];
      }
      // (2) the next tile's MFMA chain and noise block cover the LDS latency
      if (mt + 1 < NT) acc_next = row_tile<NT>(sJl, mt + 1, S, bias);
      if (mt + 1 < NT) x_next = noise_block(2u * (mt + 1) + ctr_half, tg, ctr_trial, stream, k0, k1);
      else x_next = noise_block(ctr_half, tg + 1, ctr_trial, stream, k0, k1);
      // (3) energy of s(t) and the decisions of this tile
      int d[16];
#pragma unroll
      for (int r = 0; r < kRegs; ++r) {
        int I = __float_as_int(acc[r]);  // 0x4B400000 + 2 I
        int v = I;
        if (HAS_H) {
          const int hv = sH[hoff + r];
          I += hv;
          v = I + hv;
        }
        ep += __mul24(sv[r], v);  // low 24 bits: 2^22 + 2 I (+ 4 h), below 2^23
        PIM_FENCE(ep);            // one multiply-add per term
        d[r] = I - th[r];         // >= 0  <=>  s(t+1) = +1
      }
      // sign bits of the decided registers' old spins (registers 8q + b in
      // the low nibbles, 8q + 4 + b in the high ones)
      nneg += __builtin_popcount(sw[0] & (kRegs >= 8 ? 0x88888888u : 0x08080808u)) +
              (kRegs > 8 ? __builtin_popcount(sw[1] & (kRegs >= 16 ? 0x88888888u : 0x08080808u)) : 0);
      uint32_t w[2];
#pragma unroll
      for (int q = 0; q < 2; ++q) {
        if (8 * q >= kRegs) {  // padding spins only: kept as they are
          w[q] = sw[q];
          continue;
        }
        // sign bytes of d (0xFF: s(t+1) = -1): spins 8q + b (low nibbles)
        const uint32_t lo = __builtin_amdgcn_perm((uint32_t)d[8 * q + 1], (uint32_t)d[8 * q + 0], 0x0C0C0B09u) |
                            __builtin_amdgcn_perm((uint32_t)d[8 * q + 3], (uint32_t)d[8 * q + 2], 0x0B090C0Cu);
        if (8 * q + 4 >= kRegs) {  // high nibbles are padding: keep them
          w[q] = (lo & 0x08080808u) | (sw[q] & 0xF0F0F0F0u) | (kPlusTwos & 0x0F0F0F0Fu);
          continue;
        }
        const uint32_t hi = __builtin_amdgcn_perm((uint32_t)d[8 * q + 5], (uint32_t)d[8 * q + 4], 0x0C0C0B09u) |
                            __builtin_amdgcn_perm((uint32_t)d[8 * q + 7], (uint32_t)d[8 * q + 6], 0x0B090C0Cu);
        w[q] = (lo & 0x08080808u) | (hi & 0x80808080u) | kPlusTwos;
      }
      Sn[mt] = uint2{w[0], w[1]};
      // fence the tile's results so its decisions are not sunk past the
      // next tiles' MFMA chains
      PIM_FENCE(ep);
      PIM_FENCE(Sn[mt].x);
      PIM_FENCE(Sn[mt].y);
      __builtin_amdgcn_sched_barrier(0);
    }
    // sum over decided spins of s (2^22 + 2 I + 4 h), less 2^22 sum s
    ep -= kLow24Bias * (kDecided - 2 * nneg);
    const int32_t E = -((ep + __shfl_xor(ep, 32)) / 4);  // sum s (2 I + 4 h) = 4 * (-E)
    if (E < e_best) {
      e_best = E;
      t_best = tg;
      if (live) {
        size_t off = cell * kNpad + 16 * half;
        PIM_FENCE(off);
        int8_t* dst = a.best_s + off;
#pragma unroll
        for (int mt = 0; mt < NT; ++mt) *reinterpret_cast<v4i*>(dst + 32 * mt) = i8_tile(S[mt]);
      }
    }
    if (first_hit < 0 && E <= target) first_hit = tg;
    e_cur = E;
    if (last) break;
    if ((t & 255) == 0 && __atomic_load_n(a.cancel, __ATOMIC_RELAXED) != 0) {
      done = t;  // s(t) stays the final state
      break;
    }
#pragma unroll
    for (int mt = 0; mt < NT; ++mt) S[mt] = Sn[mt];
    if (has_next) {
      // every lookup of this step precedes this write in the wave's LDS order
      stage_table(sTab, nxt, lane);
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
  }

  if (!live) return;
#pragma unroll
  for (int mt = 0; mt < NT; ++mt)
    *reinterpret_cast<v4i*>(a.final_s + cell * kNpad + 32 * mt + 16 * half) = i8_tile(S[mt]);
  if (half == 0) {
    a.e_best[cell] = e_best;
    a.t_best[cell] = t_best;
    a.first_hit[cell] = first_hit;
    a.e_final[cell] = e_cur;
    a.steps_done[cell] = done;
  }
}

template <int NT, bool HAS_H, int TAIL>
hipError_t launch_tail(const SweepArgs& a, int count, hipStream_t s) {
  const int waves = a.waves;  // 1, 2 or 4 (checked by the caller)
  const size_t lds = (size_t)NT * ((NT + 1) / 2) * 1024 + (HAS_H ? NT * 32 * 4 : 0) + (size_t)waves * kTab32Bytes;
  auto kern = sweep_mfma4_kernel<NT, HAS_H, TAIL>;
  hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  const int per_wg = 32 * waves;
  const int bpi = (a.R + per_wg - 1) / per_wg;
  const int groups = (count + kXcds - 1) / kXcds;
  const dim3 grid((unsigned)(bpi * groups * kXcds));
  hipLaunchKernelGGL(kern, grid, dim3(64 * waves), lds, s, a, bpi);
  return hipGetLastError();
}

template <int NT, bool HAS_H>
hipError_t launch_nt(const SweepArgs& a, int count, hipStream_t s) {
  const int rem = a.n - 32 * (NT - 1);  // 1 .. 32
  if (rem > 12) return launch_tail<NT, HAS_H, 16>(a, count, s);
  if (rem > 8) return launch_tail<NT, HAS_H, 12>(a, count, s);
  if (rem > 4) return launch_tail<NT, HAS_H, 8>(a, count, s);
  return launch_tail<NT, HAS_H, 4>(a, count, s);
}

template <bool HAS_H>
hipError_t launch_h(const SweepArgs& a, int count, int nt, hipStream_t s) {
  switch (nt) {
    case 1: return launch_nt<1, HAS_H>(a, count, s);
    case 2: return launch_nt<2, HAS_H>(a, count, s);
    case 3: return launch_nt<3, HAS_H>(a, count, s);
    case 4: return launch_nt<4, HAS_H>(a, count, s);
    case 5: return launch_nt<5, HAS_H>(a, count, s);
    case 6: return launch_nt<6, HAS_H>(a, count, s);
    case 7: return launch_nt<7, HAS_H>(a, count, s);
    case 8: return launch_nt<8, HAS_H>(a, count, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace

hipError_t launch_sweep_mfma4(const SweepArgs& a, int count, int nt, bool has_h, hipStream_t s) {
  if (a.npad != nt * 32 || a.trace) return hipErrorInvalidValue;
  if (a.waves != 1 && a.waves != 2 && a.waves != kWaves) return hipErrorInvalidValue;
  return has_h ? launch_h<true>(a, count, nt, s) : launch_h<false>(a, count, nt, s);
}

}  // namespace pim
