// PIMI sweep for 256 < N <= 1024 on e2m1 (FP4) matrix cores, for integer
// instances whose couplings all lie in {0, +-1, +-2, +-3, +-4, +-6}, the
// integers e2m1 represents exactly (SK-1 and unweighted Max-Cut have J in
// {0, +-1}).  The spins enter as +-2 (e2m1 0x4 / 0xC), so every product is an
// exact integer and the binary32 accumulation (|2 I| <= 2 * 32766 < 2^24, the
// bound instances are validated against) is exact in any order: the kernel
// holds twice the field of Eq. (2) exactly, compares it with doubled integer
// thresholds, and its trajectories, energies and best states are the int8
// kernel's.
// One v_mfma_f32_32x32x64_f8f6f4 on e2m1 operands issues in the cycles of one
// 32x32x32 int8 MFMA and covers twice the K, and J and the spins take 4 bits
// per value in L2 and LDS.
//
// Work split as in the int8 streamed kernel: one workgroup = 8 waves (two per
// SIMD) on 128 trials (four 32-trial column blocks) of one instance; wave w
// owns row tiles w, w + 8, w + 16, w + 24 and contracts two of them at once
// for all four column blocks, so every A fragment read from global memory
// feeds four MFMAs and every B fragment read from LDS feeds two.  One K step
// covers 64 spins: the 16-spin halves that a lane holds of two consecutive
// 32-spin tiles, so the spins a lane decides are the spins it later supplies
// to the B operand.
//
// With 4-bit spins two copies of the 128 trials' state fit in LDS (64 KB each
// at N = 1024): step t reads s(t) from one buffer and writes s(t+1) straight
// into the other, so a step needs one workgroup barrier:
//   1. contraction and decisions (Eq. (4)) of the wave's row tiles, s(t+1)
//      into the other buffer, per-trial partial energies (Eq. (1)) of s(t)
//      into this step's energy buffer;
//   -- barrier: s(t+1) and the energies of s(t) are complete --
//   2. energies reduced over the waves, best-state bookkeeping; each wave
//      copies its own rows of s(t), which only that wave ever writes.
// The step tables are double-buffered the same way.
#include <hip/hip_runtime.h>

#include <climits>
#include <cstdint>
#include <type_traits>

#include "internal.hpp"
#include "philox.hpp"
#include "e2m1.hpp"
#include "frag_stream.hpp"

namespace pim {
namespace {

using namespace e2m1;

constexpr int kWaves = 8;            // two waves per SIMD
constexpr int kCB = 4;               // 32-trial column blocks per workgroup
constexpr int kTrialsWG = 32 * kCB;  // trials per workgroup
constexpr int kXcds = 8;
constexpr int kMinTiles = PIM_MAX_N_LDS / 32 + 1;  // 9
constexpr int kMaxTiles = PIM_MAX_N / 32;          // 32

#define PIM_FENCE(v) asm volatile("" : "+v"(v))

__device__ __forceinline__ int32_t half_sum(int32_t v) {
  const auto r = __builtin_amdgcn_permlane32_swap((uint32_t)v, (uint32_t)v, false, false);
  return (int32_t)(r[0] + r[1]);
}

__device__ __forceinline__ Ctr4 noise_block(uint32_t block, int tg, uint32_t trial, uint32_t stream,
                                            uint32_t k0, uint32_t k1) {
  return philox4x32_10(Ctr4{block, (uint32_t)tg, trial, (kDomainNoise << 24) | stream}, k0, k1);
}

// Workgroup barrier for data exchanged through LDS only (outstanding global
// loads stay in flight across it).
__device__ __forceinline__ void lds_barrier() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// Spin buffer: 16-byte B-operand slot of K step p, column block c, lane l at
// (p * kCB + c) * 64 + l; row tile mt fills half mt & 1 (8 bytes) of K step mt / 2.
__device__ __forceinline__ int sb_index(int p, int c, int lane) { return (p * kCB + c) * 64 + lane; }
__device__ __forceinline__ int sb_half(int mt, int c, int lane) { return 2 * sb_index(mt >> 1, c, lane) + (mt & 1); }

// Fields of MT (1 or 2) row tiles mt0, mt0 + kWaves for the four column
// blocks over np K steps: each K step MT A fragments from global memory, four
// B fragments from LDS, MT x 4 MFMAs.  The A fragments stream through a ring
// of D slots per row tile (K step k uses slot k % D), refilled right after
// the MFMAs that read them from a clamped, always in-bounds index; the B
// fragments of the next K step are read right after the current MFMAs are
// issued; a scheduling barrier per K step keeps the compiler from hoisting
// more loads than these registers.  K step 0 is peeled so its MFMAs take a
// zero accumulator as an inline constant: inside the loop the accumulators
// would have to be zeroed by moves, one per register.
template <int MT>
__device__ __forceinline__ void rows_f4(const FragStream& gA, const v4i* sB, int lane, int mt0, int np,
                                        v16f (&acc)[MT][kCB]) {
  constexpr int D = MT == 1 ? 4 : 2;
  int fa[MT];
#pragma unroll
  for (int r = 0; r < MT; ++r) fa[r] = (mt0 + kWaves * r) * np;
  v4i ar[MT][D], b[kCB];
#pragma unroll
  for (int r = 0; r < MT; ++r)
#pragma unroll
    for (int i = 0; i < D; ++i) ar[r][i] = gA(fa[r] + i);  // np >= 5 > D
#pragma unroll
  for (int c = 0; c < kCB; ++c) b[c] = sB[sb_index(0, c, lane)];
  // K step 0
#pragma unroll
  for (int c = 0; c < kCB; ++c)
#pragma unroll
    for (int r = 0; r < MT; ++r) acc[r][c] = mfma(ar[r][0], b[c], v16f{});
#pragma unroll
  for (int r = 0; r < MT; ++r) ar[r][0] = gA(fa[r] + D);  // D < np
#pragma unroll
  for (int c = 0; c < kCB; ++c) b[c] = sB[sb_index(1, c, lane)];
  __builtin_amdgcn_sched_barrier(0);
  // K steps 1 .. np - 1: groups of D, then a tail of fewer than D
  const int nfull = 1 + (np - 1) - (np - 1) % D;
  int kt = 1;
  for (; kt < nfull; kt += D) {
#pragma unroll
    for (int i = 0; i < D; ++i) {
      const int slot = (1 + i) % D;  // K step kt + i, kt = 1 mod D
#pragma unroll
      for (int c = 0; c < kCB; ++c)
#pragma unroll
        for (int r = 0; r < MT; ++r) acc[r][c] = mfma(ar[r][slot], b[c], acc[r][c]);
      const int kf = min(kt + i + D, np - 1);
#pragma unroll
      for (int r = 0; r < MT; ++r) ar[r][slot] = gA(fa[r] + kf);
      const int kn = min(kt + i + 1, np - 1);
#pragma unroll
      for (int c = 0; c < kCB; ++c) b[c] = sB[sb_index(kn, c, lane)];
      __builtin_amdgcn_sched_barrier(0);
    }
  }
#pragma unroll
  for (int i = 0; i < D - 1; ++i) {
    if (kt + i < np) {  // uniform
      const int slot = (1 + i) % D;
#pragma unroll
      for (int c = 0; c < kCB; ++c)
#pragma unroll
        for (int r = 0; r < MT; ++r) acc[r][c] = mfma(ar[r][slot], b[c], acc[r][c]);
      if (kt + i + 1 < np) {
#pragma unroll
        for (int c = 0; c < kCB; ++c) b[c] = sB[sb_index(kt + i + 1, c, lane)];
      }
    }
  }
}

// Eq. (4) decisions and Eq. (1) energy terms of row tile mt for the four
// column blocks: s(t+1) of the tile written into the next spin buffer, the
// energy terms added to ep.  The accumulator holds 2 I exactly; tab holds the
// doubled thresholds, indexed as in the int8 kernel by u ^ s (u ^ 1 for
// s = +1, ~u for s = -1).
//   With fields (HAS_H): sH holds 2 h, the field is converted to int32, and
//   ep (int32) gathers s (2 I + 4 h).
//   Without: tab holds binary32 2 theta, the decision is one binary32
//   subtraction of exact integers, and ep (binary32) gathers (2 s)(2 I) with
//   one fused multiply-add per spin, 2 s being the old spin's e2m1 value
//   converted two at a time; a lane's step total over at most 64 spins stays
//   below 2^23, so every partial sum is exact.
template <bool HAS_H>
using EpT = typename std::conditional<HAS_H, int32_t, float>::type;

// The two e2m1 spins of byte B of w as binary32 (low nibble, high nibble).
template <int B>
__device__ __forceinline__ void spin_pair(uint32_t w, float& lo, float& hi) {
  const auto p = __builtin_amdgcn_cvt_scalef32_pk_f32_fp4(w, 1.0f, B);
  lo = p[0];
  hi = p[1];
}

template <bool HAS_H>
__device__ __forceinline__ void decide_f4(const v16f (&acc)[kCB], const uint2* sCur, uint2* sNxt,
                                          const int32_t* sH, const int32_t* tab, int mt, int lane_off, int half,
                                          uint32_t ctr_half, uint32_t ctr_trial, int tg, uint32_t stream,
                                          uint32_t k0, uint32_t k1, EpT<HAS_H> (&ep)[kCB]) {
  const int hoff = 32 * mt + 16 * half;
#pragma unroll
  for (int c = 0; c < kCB; ++c) {
    const Ctr4 x = noise_block(2u * mt + ctr_half, tg, ctr_trial + 32u * c, stream, k0, k1);
    uint32_t xw[4] = {x.x, x.y, x.z, x.w};
    const uint2 so = sCur[sb_half(mt, c, lane_off)];
    uint32_t sw[2] = {so.x, so.y};
#pragma unroll
    for (int q = 0; q < 4; ++q) PIM_FENCE(xw[q]);
    PIM_FENCE(sw[0]);
    PIM_FENCE(sw[1]);
    int sv[16], th[16];
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      sv[r] = spin_of(sw, r);
      th[r] = tab[(int)((xw[r >> 2] >> (8 * (r & 3))) & 0xFFu) ^ sv[r]];
    }
    int d[16];
    if constexpr (HAS_H) {
      int hoff_c = hoff;
      PIM_FENCE(hoff_c);
      int32_t e = ep[c];
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        int I = (int)acc[c][r];  // 2 I, exact
        const int hv = sH[hoff_c + r];
        I += hv;
        const int v = I + hv;
        e += __mul24(sv[r], v);  // |v| <= 4 * 32766 < 2^23
        PIM_FENCE(e);            // one multiply-add per term, not a multiply and an add tree
        d[r] = I - th[r];        // >= 0  <=>  s(t+1) = +1
      }
      ep[c] = e;
    } else {
      float s2[16];  // 2 s: the old spins' e2m1 values, registers 8q + b and 8q + 4 + b per byte
#pragma unroll
      for (int q = 0; q < 2; ++q) {
        spin_pair<0>(sw[q], s2[8 * q + 0], s2[8 * q + 4]);
        spin_pair<1>(sw[q], s2[8 * q + 1], s2[8 * q + 5]);
        spin_pair<2>(sw[q], s2[8 * q + 2], s2[8 * q + 6]);
        spin_pair<3>(sw[q], s2[8 * q + 3], s2[8 * q + 7]);
      }
      float e = ep[c];
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        e = __builtin_fmaf(s2[r], acc[c][r], e);                       // (2 s)(2 I), exact
        d[r] = __float_as_int(acc[c][r] - __int_as_float(th[r]));     // 2 (I - theta), exact; sign = decision
      }
      ep[c] = e;
    }
    uint32_t w[2];
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      // sign bytes of d (0xFF: s(t+1) = -1), spins 8q + b in lo, 8q + 4 + b in hi
      const uint32_t lo = __builtin_amdgcn_perm((uint32_t)d[8 * q + 1], (uint32_t)d[8 * q + 0], 0x0C0C0B09u) |
                          __builtin_amdgcn_perm((uint32_t)d[8 * q + 3], (uint32_t)d[8 * q + 2], 0x0B090C0Cu);
      const uint32_t hi = __builtin_amdgcn_perm((uint32_t)d[8 * q + 5], (uint32_t)d[8 * q + 4], 0x0C0C0B09u) |
                          __builtin_amdgcn_perm((uint32_t)d[8 * q + 7], (uint32_t)d[8 * q + 6], 0x0B090C0Cu);
      w[q] = (lo & 0x08080808u) | (hi & 0x80808080u) | kPlusTwos;
    }
    sNxt[sb_half(mt, c, lane_off)] = uint2{w[0], w[1]};
    PIM_FENCE(ep[c]);
    // one column block's decisions at a time (bounds the live temporaries)
    __builtin_amdgcn_sched_barrier(0);
  }
}

// Step table into LDS as doubled thresholds: lane l holds host entries
// 8l .. 8l + 7 (16-bit), written as eight 2 * theta, int32 with fields and
// binary32 without (|2 theta| <= 2^16: exact either way).
template <bool HAS_H>
__device__ __forceinline__ void stage_table(int32_t* dst, uint4 v, int lane) {
  const uint32_t w[4] = {v.x, v.y, v.z, v.w};
  int32_t o[8];
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    o[2 * q] = (int32_t)(w[q] << 16) >> 15;               // 2 * sign-extended low half
    o[2 * q + 1] = (int32_t)(w[q] & 0xFFFF0000u) >> 15;   // 2 * sign-extended high half
    if (!HAS_H) {
      o[2 * q] = __float_as_int((float)o[2 * q]);
      o[2 * q + 1] = __float_as_int((float)o[2 * q + 1]);
    }
  }
  reinterpret_cast<int4*>(dst)[2 * lane] = int4{o[0], o[1], o[2], o[3]};
  reinterpret_cast<int4*>(dst)[2 * lane + 1] = int4{o[4], o[5], o[6], o[7]};
}

// One workgroup's run: trial block tblk (128 trials) of instance inst.
template <int RPW, bool HAS_H>
__device__ __forceinline__ void big4_body(const SweepArgs& a, int nt, int inst, int tblk) {
  extern __shared__ __align__(16) unsigned char lds[];
  const int npad = nt * 32;
  const int np = (nt + 1) >> 1;  // K steps of 64 spins
  const int buf = np * kCB * 64;  // 16-byte slots per spin buffer
  // LDS: spins [2][np][kCB][64] x 16 B | tables [2] x 2 KB | energy partials
  // [2][kWaves][kCB][32] | per-trial t_best, first_hit, e_cur [3][kCB][32] |
  // cancel flag | 2 h
  v4i* sB = reinterpret_cast<v4i*>(lds);
  unsigned char* rest = lds + (size_t)2 * buf * 16;
  int32_t* sTab = reinterpret_cast<int32_t*>(rest);
  int32_t* sE = reinterpret_cast<int32_t*>(rest + 2 * kTab32Bytes);
  int32_t* sStat = sE + 2 * kWaves * kCB * 32;
  int32_t* sFlag = sStat + 3 * kCB * 32;
  int32_t* sH = sFlag + 4;

  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  const int col = lane & 31;
  const int half = lane >> 5;
  const int trial0 = tblk * kTrialsWG + col;
  const size_t cell0 = (size_t)inst * a.R + trial0;
  const bool writer = wave == 0 && half == 0;
  const uint32_t stream = a.inst_stream[inst];
  const int cls = a.inst_class[inst];
  const uint4* gTab4 = reinterpret_cast<const uint4*>(a.thtab + (size_t)cls * a.T * kTabEntries);
  const int32_t target = a.target ? a.target[inst] : INT_MIN;
  const uint32_t k0 = a.k0, k1 = a.k1;
  // the instance's A fragments (row tile mt, K step p, lane l at
  // fragment mt * np + p; at most 32 * 16 fragments of 1 KB)
  const FragStream gA(a.jfrag + (size_t)inst * nt * np * 1024, (uint32_t)(nt * np * 1024), lane);

  if (HAS_H)
    for (int i = threadIdx.x; i < npad; i += 64 * kWaves) sH[i] = 2 * a.h[(size_t)inst * npad + i];
  // s(0) into buffer 0: each wave its own row tiles
  uint2* sB2 = reinterpret_cast<uint2*>(sB);
#pragma unroll
  for (int j = 0; j < RPW; ++j) {
    const int mt = wave + kWaves * j;
    if (mt >= nt) break;  // uniform
#pragma unroll
    for (int c = 0; c < kCB; ++c) {
      v4i v;
      if (a.init) {
        v = (trial0 + 32 * c < a.R) ? *reinterpret_cast<const v4i*>(a.init + (cell0 + 32 * c) * npad + 32 * mt + 16 * half)
                    : v4i{0x01010101, 0x01010101, 0x01010101, 0x01010101};
      } else {
        const Ctr4 x = philox4x32_10(Ctr4{(uint32_t)(2 * mt + half), 0u, (uint32_t)(trial0 + 32 * c),
                                          (kDomainInit << 24) | stream}, k0, k1);
        v = v4i{(int)spins_from_bits(x.x), (int)spins_from_bits(x.y), (int)spins_from_bits(x.z),
                (int)spins_from_bits(x.w)};
      }
      sB2[sb_half(mt, c, lane)] = nib_tile(v);
    }
  }
  // odd tile count: the second half of the last K step has no spins (its
  // couplings are zero); give it +1 in both buffers
  if ((nt & 1) && wave == kWaves - 1)
#pragma unroll
    for (int c = 0; c < kCB; ++c) {
      sB2[sb_half(nt, c, lane)] = uint2{kPlusTwos, kPlusTwos};
      sB2[2 * buf + sb_half(nt, c, lane)] = uint2{kPlusTwos, kPlusTwos};
    }
  // table of step 0 into table buffer 0; the next one waits in registers
  uint4 nxt = uint4{0, 0, 0, 0};
  if (wave == 0) {
    stage_table<HAS_H>(sTab, gTab4[lane], lane);
    nxt = gTab4[(size_t)min(1, a.T - 1) * 64 + lane];
  }
  if (threadIdx.x == 0) sFlag[0] = 0;
  if (writer)
#pragma unroll
    for (int c = 0; c < kCB; ++c) {
      sStat[(0 * kCB + c) * 32 + col] = -1;  // t_best
      sStat[(1 * kCB + c) * 32 + col] = -1;  // first_hit
      sStat[(2 * kCB + c) * 32 + col] = 0;   // e_cur
    }
  __syncthreads();

  int32_t e_best[kCB];
#pragma unroll
  for (int c = 0; c < kCB; ++c) e_best[c] = INT_MAX;
  int done = a.T;
  int t = 0;
  const int rw = (nt - wave + kWaves - 1) / kWaves;  // row tiles of this wave (>= 1: nt >= 9 > wave)
  for (;; ++t) {
    const int tg = a.start_step + t;
    const int cur = t & 1;
    // the table of step t+1 into the other table buffer (last read in step
    // t-1, before its barrier), then the fetch of the one after
    if (wave == 0) {
      stage_table<HAS_H>(sTab + (cur ^ 1) * kTabEntries, nxt, lane);
      nxt = gTab4[(size_t)min(t + 2, a.T - 1) * 64 + lane];
    }
    const int32_t* tab = sTab + cur * kTabEntries + kNoiseVals;
    const v4i* sCur = sB + cur * buf;
    const uint2* sCur2 = reinterpret_cast<const uint2*>(sCur);
    uint2* sNxt2 = sB2 + (cur ^ 1) * 2 * buf;
    EpT<HAS_H> ep[kCB];
#pragma unroll
    for (int c = 0; c < kCB; ++c) ep[c] = 0;
    uint32_t ctr_half = (uint32_t)half, ctr_trial = (uint32_t)trial0;
    int lane_off = lane;
    PIM_FENCE(ctr_half);
    PIM_FENCE(ctr_trial);
    PIM_FENCE(lane_off);
    // ---- phase 1: contraction and decisions, s(t+1) into the other buffer ----
#pragma unroll
    for (int g = 0; g < (RPW + 1) / 2; ++g) {
      const int j0 = 2 * g;
      if (j0 >= rw) break;  // uniform
      const int mt0 = wave + kWaves * j0;
      if (j0 + 1 < rw) {
        v16f acc[2][kCB];
        rows_f4<2>(gA, sCur, lane_off, mt0, np, acc);
        decide_f4<HAS_H>(acc[0], sCur2, sNxt2, sH, tab, mt0, lane_off, half, ctr_half, ctr_trial, tg, stream, k0,
                         k1, ep);
        decide_f4<HAS_H>(acc[1], sCur2, sNxt2, sH, tab, mt0 + kWaves, lane_off, half, ctr_half, ctr_trial, tg,
                         stream, k0, k1, ep);
      } else {
        v16f acc[1][kCB];
        rows_f4<1>(gA, sCur, lane_off, mt0, np, acc);
        decide_f4<HAS_H>(acc[0], sCur2, sNxt2, sH, tab, mt0, lane_off, half, ctr_half, ctr_trial, tg, stream, k0,
                         k1, ep);
      }
    }
    // per-trial partial energies of s(t) over this wave's rows
#pragma unroll
    for (int c = 0; c < kCB; ++c) {
      const int32_t epc = half_sum((int32_t)ep[c]);  // binary32 totals are exact integers below 2^23
      if (half == 0) sE[((cur * kWaves + wave) * kCB + c) * 32 + col] = epc;
    }
    if (threadIdx.x == 0 && (t & 255) == 0 && t < a.T)
      sFlag[0] = __atomic_load_n(a.cancel, __ATOMIC_RELAXED) != 0 ? 1 : 0;
    lds_barrier();  // s(t+1), the table of step t+1 and the energies of s(t) are complete
    // ---- phase 2: energies and bookkeeping of s(t) ----
#pragma unroll
    for (int c = 0; c < kCB; ++c) {
      int32_t tot = 0;
#pragma unroll
      for (int w = 0; w < kWaves; ++w) tot += sE[((cur * kWaves + w) * kCB + c) * 32 + col];
      // tot = 2 sum_i s_i (I_i + 2 h_i) with fields, 4 sum_i s_i I_i without
      const int32_t E = HAS_H ? -(tot / 4) : -(tot / 8);
      if (E < e_best[c]) {
        e_best[c] = E;
        if (writer) sStat[(0 * kCB + c) * 32 + col] = tg;
        if (trial0 + 32 * c < a.R) {
          size_t off = (cell0 + 32 * c) * npad + 16 * half;
          PIM_FENCE(off);
          int8_t* dst = a.best_s + off;
#pragma unroll
          for (int j = 0; j < RPW; ++j) {
            const int mt = wave + kWaves * j;
            if (mt < nt) *reinterpret_cast<v4i*>(dst + 32 * mt) = i8_tile(sCur2[sb_half(mt, c, lane)]);
          }
        }
      }
      if (writer) {
        if (sStat[(1 * kCB + c) * 32 + col] < 0 && E <= target) sStat[(1 * kCB + c) * 32 + col] = tg;
        sStat[(2 * kCB + c) * 32 + col] = E;
      }
    }
    if (t == a.T) break;  // uniform: s(T) is in buffer T & 1
    if ((t & 255) == 0 && sFlag[0] != 0) {  // uniform: written before the barrier
      done = t;  // s(t) stays the final state
      break;
    }
  }
  // final state: s(t) in buffer t & 1, this wave's own rows
  const uint2* sFin = sB2 + (t & 1) * 2 * buf;
#pragma unroll
  for (int c = 0; c < kCB; ++c) {
    if (!(trial0 + 32 * c < a.R)) continue;
#pragma unroll
    for (int j = 0; j < RPW; ++j) {
      const int mt = wave + kWaves * j;
      if (mt < nt)
        *reinterpret_cast<v4i*>(a.final_s + (cell0 + 32 * c) * npad + 32 * mt + 16 * half) =
            i8_tile(sFin[sb_half(mt, c, lane)]);
    }
    if (writer) {
      a.e_best[cell0 + 32 * c] = e_best[c];
      a.t_best[cell0 + 32 * c] = sStat[(0 * kCB + c) * 32 + col];
      a.first_hit[cell0 + 32 * c] = sStat[(1 * kCB + c) * 32 + col];
      a.e_final[cell0 + 32 * c] = sStat[(2 * kCB + c) * 32 + col];
      a.steps_done[cell0 + 32 * c] = done;
    }
  }
}

template <int RPW, bool HAS_H>
__global__ __launch_bounds__(64 * kWaves, 2) void sweep_big4_kernel(SweepArgs a, int nt, int blocks_per_inst) {
  // workgroup -> (instance, trial block): the blocks of instance k all have
  // linear ids congruent to k modulo the XCD count (hardware dispatch sends
  // consecutive workgroups to consecutive XCDs), so they share one L2
  const int lin = blockIdx.x;
  const int inst = (lin % kXcds) + kXcds * ((lin / kXcds) / blocks_per_inst);
  const int tblk = (lin / kXcds) % blocks_per_inst;
  if (inst >= a.count) return;  // whole workgroup: before any barrier
  big4_body<RPW, HAS_H>(a, nt, inst, tblk);
}

// Several batches of different N in one launch: workgroup b runs work item
// work[b] = (part, instance, trial block) with that part's arguments.  The
// host orders the items so that workgroups 8k + x all run on XCD x, each
// instance's blocks on one XCD, and each XCD's items longest first.
template <bool HAS_H>
__global__ __launch_bounds__(64 * kWaves, 2) void sweep_big4_multi_kernel(const MultiPart* parts, const int4* work,
                                                                          int nwork, MultiRun run) {
  if ((int)blockIdx.x >= nwork) return;
  const int4 item = work[blockIdx.x];
  if (item.x < 0) return;  // padding item: whole workgroup, before any barrier
  SweepArgs a = parts[item.x].a;
  const int nt = parts[item.x].nt;
  a.k0 = run.k0;
  a.k1 = run.k1;
  a.T = run.T;
  a.start_step = run.start_step;
  if (!run.use_target) a.target = nullptr;
  big4_body<kMaxTiles / kWaves, HAS_H>(a, nt, item.y, item.z);
}

size_t big4_lds_bytes(int nt, bool has_h) {
  const size_t np = (size_t)(nt + 1) / 2;
  return 2 * np * kCB * 1024 + 2 * kTab32Bytes + (size_t)(2 * kWaves + 3) * kCB * 32 * 4 + 16 +
         (has_h ? (size_t)nt * 32 * 4 : 0);
}

template <int RPW, bool HAS_H>
hipError_t launch_rpw(const SweepArgs& a, int count, int nt, hipStream_t s) {
  const size_t lds = big4_lds_bytes(nt, HAS_H);
  auto kern = sweep_big4_kernel<RPW, HAS_H>;
  hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  const int bpi = (a.R + kTrialsWG - 1) / kTrialsWG;
  const int groups = (count + kXcds - 1) / kXcds;
  const dim3 grid((unsigned)(bpi * groups * kXcds));
  hipLaunchKernelGGL(kern, grid, dim3(64 * kWaves), lds, s, a, nt, bpi);
  return hipGetLastError();
}

template <bool HAS_H>
hipError_t launch_h(const SweepArgs& a, int count, int nt, hipStream_t s) {
  switch ((nt + kWaves - 1) / kWaves) {  // row tiles per wave
    case 2: return launch_rpw<2, HAS_H>(a, count, nt, s);
    case 3: return launch_rpw<3, HAS_H>(a, count, nt, s);
    case 4: return launch_rpw<4, HAS_H>(a, count, nt, s);
    default: return hipErrorInvalidValue;
  }
}

// e2m1 code of an integer coupling in {0, +-1, +-2, +-3, +-4, +-6}; 0xFF otherwise.
uint8_t e2m1_code(int v) {
  const int m = v < 0 ? -v : v;
  uint8_t c;
  switch (m) {
    case 0: return 0;  // +0
    case 1: c = 0x2; break;
    case 2: c = 0x4; break;
    case 3: c = 0x5; break;
    case 4: c = 0x6; break;
    case 6: c = 0x7; break;
    default: return 0xFF;
  }
  return (uint8_t)(v < 0 ? c | 0x8 : c);
}

}  // namespace

bool f4_couplings(const int8_t* J, size_t count) {
  for (size_t i = 0; i < count; ++i)
    if (e2m1_code(J[i]) == 0xFF) return false;
  return true;
}

size_t f4_frag_bytes(int nt) { return (size_t)nt * ((nt + 1) / 2) * 1024; }

// A fragment of row tile mt and K step p, lane l = 32 g + m, element e (nibble
// e % 8 of word e / 8, low nibble first): physical row m carries spin
// 32 mt + 16 ((m / 4) % 2) + 4 (m / 8) + m % 4 (the int8 kernel's order), and
// element e carries spin 32 (2p + e / 16) + 16 g + r with, for n = e % 8 and
// q = (e / 8) % 2, r = 8q + 4 (n % 2) + n / 2: the register order in which
// the kernel packs a tile's decided spins.
void pack_f4_fragments(const int8_t* J, int n, int nt, uint8_t* out) {
  const int np = (nt + 1) / 2;
  for (int mt = 0; mt < nt; ++mt)
    for (int p = 0; p < np; ++p)
      for (int l = 0; l < 64; ++l) {
        const int m = l & 31, g = l >> 5;
        const int row = 32 * mt + 16 * ((m >> 2) & 1) + 4 * (m >> 3) + (m & 3);
        uint8_t* dst = out + (((size_t)mt * np + p) * 64 + l) * 16;
        for (int i = 0; i < 16; ++i) dst[i] = 0;
        for (int e = 0; e < 32; ++e) {
          const int nn = e & 7, q = (e >> 3) & 1;
          const int r = 8 * q + 4 * (nn & 1) + (nn >> 1);
          const int colj = 32 * (2 * p + (e >> 4)) + 16 * g + r;
          const int v = (row < n && colj < n) ? J[(size_t)row * n + colj] : 0;
          dst[e >> 1] |= (uint8_t)(e2m1_code(v) << (4 * (e & 1)));
        }
      }
}

template <bool HAS_H>
hipError_t launch_multi(const MultiPart* d_parts, const int4* d_work, int nwork, int nt_max, const MultiRun& run,
                        hipStream_t s) {
  const size_t lds = big4_lds_bytes(nt_max, HAS_H);
  auto kern = sweep_big4_multi_kernel<HAS_H>;
  hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(kern), hipFuncAttributeMaxDynamicSharedMemorySize,
                                     (int)lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(kern, dim3((unsigned)nwork), dim3(64 * kWaves), lds, s, d_parts, d_work, nwork, run);
  return hipGetLastError();
}

hipError_t launch_sweep_big4_multi(const MultiPart* d_parts, const int4* d_work, int nwork, int nt_max, bool has_h,
                                   const MultiRun& run, hipStream_t s) {
  if (nwork < 1 || nt_max < kMinTiles || nt_max > kMaxTiles) return hipErrorInvalidValue;
  return has_h ? launch_multi<true>(d_parts, d_work, nwork, nt_max, run, s)
               : launch_multi<false>(d_parts, d_work, nwork, nt_max, run, s);
}

// Relative time of one workgroup-step at nt row tiles: the waves of a SIMD
// (w and w + 4) run their tiles' contractions (4 MFMAs per tile and K step)
// and decisions (4 blocks of 16 per tile) one after the other, and the
// workgroup waits at every step for its busiest SIMD.
double big4_step_cost(int nt) {
  const int np = (nt + 1) / 2;
  int simd_tiles = 0;
  for (int w = 0; w < kWaves / 2; ++w) {
    const int t = (nt - w + kWaves - 1) / kWaves + (nt - w - kWaves / 2 + kWaves - 1) / kWaves;
    simd_tiles = t > simd_tiles ? t : simd_tiles;
  }
  return simd_tiles * (128.0 * np + 2660.0) + 3000.0;
}

hipError_t launch_sweep_big4(const SweepArgs& a, int count, int nt, bool has_h, hipStream_t s) {
  if (a.npad != nt * 32 || nt < kMinTiles || nt > kMaxTiles || a.T < 1 || count < 1 || a.R < 1)
    return hipErrorInvalidValue;
  return has_h ? launch_h<true>(a, count, nt, s) : launch_h<false>(a, count, nt, s);
}

}  // namespace pim
