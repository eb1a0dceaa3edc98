// PIMI sweep on int8 MFMA for 256 < N <= 1024, where N^2 bytes of couplings no
// longer fit in LDS.
//
// One workgroup = 4 waves sharing one block of 32 trials of one instance.
// Wave w owns the row tiles mt = w, w + 4, w + 8, ...; each row tile's field
// (Eq. (2)) is a chain of NT v_mfma_i32_32x32x32_i8 over the K tiles, with the
// A fragments (the same permuted fragment order as the LDS-resident kernel)
// read from global memory (L2 / the last-level cache) and the B operand, the
// current spins of all 32 trials, read from an LDS spin buffer that the four
// waves fill together: each wave writes the new spins of its own row tiles
// into the other half of a double buffer, and one workgroup barrier per step
// makes s(t+1) complete.  Decisions (Eq. (4)) use the same integer
// (u, s) threshold table, shared by the workgroup and double-buffered in LDS;
// the energy (Eq. (1)) of each trial is reduced over the waves in LDS.
//
// Workgroups are mapped so that all blocks of one instance run on one XCD
// (hardware dispatch sends consecutive workgroups to consecutive XCDs), which
// keeps the instance's couplings in that XCD's L2.
#include <hip/hip_runtime.h>

#include <climits>
#include <cstdint>

#include "internal.hpp"
#include "philox.hpp"

namespace pim {
namespace {

typedef int v4i __attribute__((ext_vector_type(4)));
typedef int v16i __attribute__((ext_vector_type(16)));

constexpr int kWaves = 4;
constexpr int kXcds = 8;
constexpr int kTabBytes = kTabEntries * 2;

#define PIM_FENCE(v) asm volatile("" : "+v"(v))

__device__ __forceinline__ int spins_from_bits(uint32_t w) {
  return (int)(0xFFFFFFFFu - 0xFEu * ((w >> 7) & 0x01010101u));
}

__device__ __forceinline__ Ctr4 noise_block(uint32_t block, int tg, uint32_t trial, uint32_t stream,
                                            uint32_t k0, uint32_t k1) {
  return philox4x32_10(Ctr4{block, (uint32_t)tg, trial, (kDomainNoise << 24) | stream}, k0, k1);
}

// Field of row tile mt: A fragments from global memory, B from the LDS spin
// buffer (tile kt of lane l at (kt * 64 + l)).
template <int NT>
__device__ __forceinline__ v16i big_row_tile(const v4i* __restrict__ gA, const v4i* sB, int lane, int mt) {
  v16i acc = v16i{};
  const v4i* a = gA + (size_t)mt * NT * 64 + lane;
  // partial unroll: a full unroll lets the compiler hoist all 2 NT operand
  // loads ahead of the chain, which does not fit the register file at large NT
#pragma unroll 4
  for (int kt = 0; kt < NT; ++kt) acc = __builtin_amdgcn_mfma_i32_32x32x32_i8(a[kt * 64], sB[kt * 64 + lane], acc, 0, 0, 0);
  return acc;
}

template <int NT, bool HAS_H>
__global__ __launch_bounds__(64 * kWaves) void sweep_big_kernel(SweepArgs a, int blocks_per_inst) {
  extern __shared__ __align__(16) unsigned char lds[];
  constexpr int kNpad = NT * 32;
  constexpr int kPerWave = NT / kWaves;  // row tiles per wave
  // LDS: spins [2][NT][64] x 16 B | table [2] x 1 KB | energy partials
  // [2][4][32] | cancel flag | h.  Spins, tables and partials are double-
  // buffered by step parity, so one barrier per step orders everything: a
  // buffer is rewritten two steps after it was read, and every wave has
  // passed the intervening barrier.
  v4i* sB = reinterpret_cast<v4i*>(lds);
  int16_t* sTab = reinterpret_cast<int16_t*>(lds + 2 * NT * 1024);
  int32_t* sE = reinterpret_cast<int32_t*>(lds + 2 * NT * 1024 + 2 * kTabBytes);
  int32_t* sFlag = sE + 2 * kWaves * 32;
  int32_t* sH = sFlag + 4;

  // workgroup -> (instance, trial block): the blocks of instance k all have
  // linear ids congruent to k modulo the XCD count
  const int lin = blockIdx.x;
  const int inst = (lin % kXcds) + kXcds * ((lin / kXcds) / blocks_per_inst);
  const int tblk = (lin / kXcds) % blocks_per_inst;
  if (inst >= a.count) return;  // whole workgroup: before any barrier
  const int wave = threadIdx.x >> 6;
  const int lane = threadIdx.x & 63;
  const int col = lane & 31;
  const int half = lane >> 5;
  const int trial = tblk * 32 + col;
  const bool live = trial < a.R;
  const size_t cell = (size_t)inst * a.R + trial;
  const uint32_t stream = a.inst_stream[inst];
  const int cls = a.inst_class[inst];
  const uint4* gTab4 = reinterpret_cast<const uint4*>(a.thtab + (size_t)cls * a.T * kTabEntries);
  const int32_t target = a.target ? a.target[inst] : INT_MIN;
  const uint32_t k0 = a.k0, k1 = a.k1;
  const v4i* gA = reinterpret_cast<const v4i*>(a.jfrag + (size_t)inst * NT * NT * 1024);

  if (HAS_H)
    for (int i = threadIdx.x; i < kNpad; i += 64 * kWaves) sH[i] = a.h[(size_t)inst * kNpad + i];
  // s(0): each wave its own row tiles
#pragma unroll
  for (int j = 0; j < kPerWave; ++j) {
    const int mt = wave + kWaves * j;
    v4i v;
    if (a.init) {
      v = live ? *reinterpret_cast<const v4i*>(a.init + cell * kNpad + 32 * mt + 16 * half)
               : v4i{0x01010101, 0x01010101, 0x01010101, 0x01010101};
    } else {
      const Ctr4 x = philox4x32_10(Ctr4{(uint32_t)(2 * mt + half), 0u, (uint32_t)trial,
                                        (kDomainInit << 24) | stream}, k0, k1);
      v = v4i{spins_from_bits(x.x), spins_from_bits(x.y), spins_from_bits(x.z), spins_from_bits(x.w)};
    }
    sB[mt * 64 + lane] = v;
  }
  if (wave == 0) reinterpret_cast<uint4*>(sTab)[lane] = gTab4[lane];
  if (threadIdx.x == 0) sFlag[0] = 0;
  __syncthreads();

  int32_t e_best = INT_MAX, t_best = -1, first_hit = -1, e_cur = 0;
  int done = a.T;
  int cur = 0;
  for (int t = 0;; ++t) {
    const int tg = a.start_step + t;
    const v4i* sCur = sB + cur * NT * 64;
    v4i* sNxt = sB + (cur ^ 1) * NT * 64;
    const int16_t* tab = sTab + (t & 1) * kTabEntries + kNoiseVals;
    // wave 0 fetches the table of step t+1 (written before this step's barrier)
    uint4 nxt = uint4{0, 0, 0, 0};
    if (wave == 0) nxt = gTab4[(size_t)min(t + 1, a.T - 1) * 64 + lane];
    int32_t ep = 0;
    Ctr4 x_next = noise_block(2u * wave + half, tg, (uint32_t)trial, stream, k0, k1);
    v16i acc_next = big_row_tile<NT>(gA, sCur, lane, wave);
#pragma unroll
    for (int j = 0; j < kPerWave; ++j) {
      const int mt = wave + kWaves * j;
      const v16i acc = acc_next;
      uint32_t xw[4] = {x_next.x, x_next.y, x_next.z, x_next.w};
      const v4i cv = sCur[mt * 64 + lane];
      uint32_t bw[4] = {(uint32_t)cv[0], (uint32_t)cv[1], (uint32_t)cv[2], (uint32_t)cv[3]};
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        PIM_FENCE(xw[q]);
        PIM_FENCE(bw[q]);
      }
      int th[16];
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int sv = (int)(int8_t)(bw[r >> 2] >> (8 * (r & 3)));
        th[r] = tab[(int)((xw[r >> 2] >> (8 * (r & 3))) & 0xFFu) ^ sv];
      }
      if (j + 1 < kPerWave) {
        acc_next = big_row_tile<NT>(gA, sCur, lane, mt + kWaves);
        x_next = noise_block(2u * (mt + kWaves) + half, tg, (uint32_t)trial, stream, k0, k1);
      }
      const int hoff = 32 * mt + 16 * half;
      v4i o;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        int d[4];
#pragma unroll
        for (int b = 0; b < 4; ++b) {
          const int r = 4 * q + b;
          const int sv = (int)(int8_t)(bw[q] >> (8 * b));
          int I = acc[r];
          int v = I;
          if (HAS_H) {
            const int hv = sH[hoff + r];
            I += hv;
            v = I + hv;
          }
          ep += __mul24(sv, v);
          d[b] = I - th[r];
        }
        const uint32_t p01 = __builtin_amdgcn_perm((uint32_t)d[1], (uint32_t)d[0], 0x0C0C0B09u);
        const uint32_t p23 = __builtin_amdgcn_perm((uint32_t)d[3], (uint32_t)d[2], 0x0B090C0Cu);
        o[q] = (int)(p01 | p23 | 0x01010101u);
      }
      sNxt[mt * 64 + lane] = o;
      PIM_FENCE(ep);
      __builtin_amdgcn_sched_barrier(0);
    }
    // per-trial partial energy of this wave's rows (both lane halves)
    const int32_t epc = ep + __shfl_xor(ep, 32);
    int32_t* sEt = sE + (t & 1) * kWaves * 32;
    if (half == 0) sEt[wave * 32 + col] = epc;
    if (wave == 0) reinterpret_cast<uint4*>(sTab + ((t + 1) & 1) * kTabEntries)[lane] = nxt;
    if (threadIdx.x == 0 && (t & 255) == 0 && t < a.T)
      sFlag[0] = __atomic_load_n(a.cancel, __ATOMIC_RELAXED) != 0 ? 1 : 0;
    __syncthreads();  // s(t+1), the energies of s(t) and the next table are complete
    int32_t tot = 0;
#pragma unroll
    for (int w = 0; w < kWaves; ++w) tot += sEt[w * 32 + col];
    const int32_t E = -(tot / 2);
    if (E < e_best) {
      e_best = E;
      t_best = tg;
      if (live) {
#pragma unroll
        for (int j = 0; j < kPerWave; ++j) {
          const int mt = wave + kWaves * j;
          *reinterpret_cast<v4i*>(a.best_s + cell * kNpad + 32 * mt + 16 * half) = sCur[mt * 64 + lane];
        }
      }
    }
    if (first_hit < 0 && E <= target) first_hit = tg;
    e_cur = E;
    if (t == a.T) break;  // uniform
    const bool stop = (t & 255) == 0 && sFlag[0] != 0;  // uniform: read after the barrier
    if (stop) {
      done = t;
      break;
    }
    cur ^= 1;
  }
  // final state: s(t) of the last step (in sCur)
  if (live) {
    const v4i* sCur = sB + cur * NT * 64;
#pragma unroll
    for (int j = 0; j < kPerWave; ++j) {
      const int mt = wave + kWaves * j;
      *reinterpret_cast<v4i*>(a.final_s + cell * kNpad + 32 * mt + 16 * half) = sCur[mt * 64 + lane];
    }
    if (wave == 0 && half == 0) {
      a.e_best[cell] = e_best;
      a.t_best[cell] = t_best;
      a.first_hit[cell] = first_hit;
      a.e_final[cell] = e_cur;
      a.steps_done[cell] = done;
    }
  }
}

template <int NT, bool HAS_H>
hipError_t launch_nt(const SweepArgs& a, int count, hipStream_t s) {
  const size_t lds = 2 * (size_t)NT * 1024 + 2 * kTabBytes + (2 * kWaves * 32 + 4) * 4 + (HAS_H ? NT * 32 * 4 : 0);
  auto kern = sweep_big_kernel<NT, HAS_H>;
  hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  const int bpi = (a.R + 31) / 32;
  const int groups = (count + kXcds - 1) / kXcds;
  const dim3 grid((unsigned)(bpi * groups * kXcds));
  hipLaunchKernelGGL(kern, grid, dim3(64 * kWaves), lds, s, a, bpi);
  return hipGetLastError();
}

template <bool HAS_H>
hipError_t launch_h(const SweepArgs& a, int count, int nt, hipStream_t s) {
  switch (nt) {
    case 12: return launch_nt<12, HAS_H>(a, count, s);
    case 16: return launch_nt<16, HAS_H>(a, count, s);
    case 20: return launch_nt<20, HAS_H>(a, count, s);
    case 24: return launch_nt<24, HAS_H>(a, count, s);
    case 28: return launch_nt<28, HAS_H>(a, count, s);
    case 32: return launch_nt<32, HAS_H>(a, count, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace

int big_tiles(int n) { return kWaves * ((n + 32 * kWaves - 1) / (32 * kWaves)); }

hipError_t launch_sweep_big(const SweepArgs& a, int count, int nt, bool has_h, hipStream_t s) {
  if (a.npad != nt * 32 || nt % kWaves != 0 || a.T < 1) return hipErrorInvalidValue;
  return has_h ? launch_h<true>(a, count, nt, s) : launch_h<false>(a, count, nt, s);
}

}  // namespace pim
