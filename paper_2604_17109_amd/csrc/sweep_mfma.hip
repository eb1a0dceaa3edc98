// Persistent PIMI sweep on int8 MFMA (gfx950).
//
// One workgroup holds one instance's couplings in LDS; each wave owns 32
// trials (the MFMA N dimension) and every spin row of the instance, so a whole
// update step (Eq. (2) contraction, Eq. (4) decision, Eq. (1) energy) happens
// inside the wave with no barrier:
//
//   I[Npad x 32] = J'[Npad x Npad] . S[Npad x 32]     v_mfma_i32_32x32x32_i8
//
// Layout.  With 32x32x32 int8 MFMA, lane l (column n = l % 32, half
// hh = l / 32) receives output rows 8*(r/4) + 4*hh + r%4 in register r, and
// supplies B-operand bytes p = 0..15 of K-slot (hh, p).  The spin index is
// permuted so that register r of half hh of row tile mt is spin
// 32*mt + 16*hh + r, and K-slot (hh, p) of K tile kt is spin 32*kt + 16*hh + p.
// Then the new spin of output register r is exactly B byte r of the same lane:
// the C -> B hand-off of the next step never leaves the lane, and the 16 spins a
// lane-half owns in a tile are one Philox block (16 bytes) of the noise.
//
// Decision.  The host compiles step t into a table over (noise index u, sign
// of s_i(t)) of integer field thresholds; s_i(t+1) = +1 iff I_i >= tab[u ^ s]
// (index u ^ 1 for s = +1 and ~u for s = -1, both relative to the table's
// centre, so the two halves are disjoint).
// Each wave keeps that 1 KB table in LDS and streams the next step's copy from
// global memory into registers while it works on the current one.
#include <hip/hip_runtime.h>

#include <climits>
#include <cstdint>

#include "internal.hpp"
#include "philox.hpp"

namespace pim {
namespace {

typedef int v4i __attribute__((ext_vector_type(4)));
typedef int v16i __attribute__((ext_vector_type(16)));

constexpr int kWaves = 4;                 // most waves (32-trial blocks) per workgroup
constexpr int kXcds = 8;                  // XCDs of the device (workgroup placement)
constexpr int kTabBytes = kTabEntries * 2;  // 1 KB per step table
static_assert(kTabBytes == 64 * 16, "one 16-byte chunk per lane");

// +1 where the byte's top bit (u >= 128) is set, -1 elsewhere.
__device__ __forceinline__ int spins_from_bits(uint32_t w) {
  return (int)(0xFFFFFFFFu - 0xFEu * ((w >> 7) & 0x01010101u));
}

// One Philox block of noise: counter (block, step, trial, stream) in the NOISE
// domain; its 16 bytes are the noise indices of 16 consecutive spins.
__device__ __forceinline__ Ctr4 noise_block(uint32_t block, int tg, uint32_t trial, uint32_t stream,
                                            uint32_t k0, uint32_t k1) {
  return philox4x32_10(Ctr4{block, (uint32_t)tg, trial, (kDomainNoise << 24) | stream}, k0, k1);
}

// Ordering fence for the instruction selector: the value passes through an
// empty volatile asm, so arithmetic that depends on it cannot be hoisted above
// this point (scheduling barriers only bind the later machine scheduler).
// Emits no instruction.
#define PIM_FENCE(v) asm volatile("" : "+v"(v))

// I for row tile mt of the wave's CB x 32 trials: NT chained int8 MFMAs per
// column block over the K tiles; each A fragment is read from LDS once and
// used by every column block.
template <int NT, int CB>
__device__ __forceinline__ void mfma_row_tile(const v4i* sJl, int mt, const v4i (&B)[CB][NT], v16i (&acc)[CB]) {
#pragma unroll
  for (int c = 0; c < CB; ++c) acc[c] = v16i{};
#pragma unroll
  for (int kt = 0; kt < NT; ++kt) {
    const v4i A = sJl[(mt * NT + kt) * 64];
#pragma unroll
    for (int c = 0; c < CB; ++c) acc[c] = __builtin_amdgcn_mfma_i32_32x32x32_i8(A, B[c][kt], acc[c], 0, 0, 0);
  }
}

// Each wave owns CB blocks of 32 trials.  Two independent blocks give the
// in-order issue of one wave per SIMD enough independent work to keep the
// vector ALU busy while MFMA chains and LDS lookups are in flight.
//
// TAIL (4, 8, 12 or 16) is how many of a lane's 16 registers of the last row
// tile carry spins below N in the lower lane half, rounded up to 4: spins
// 32 (NT - 1) + r for r < N - 32 (NT - 1).  Decisions and energy terms are
// skipped for the registers past it.  Those hold padding spins only (zero
// rows and columns of J, so their fields are 0 and they never enter another
// spin's field); they keep their initial values.  In the upper lane half the
// same registers hold spins 32 (NT - 1) + 16 + r, which are padding whenever
// TAIL < 16.
template <int NT, int CB, bool HAS_H, bool RECORD, int TAIL>
__global__ __launch_bounds__(64 * kWaves, 3) void sweep_mfma_kernel(SweepArgs a, int blocks_per_inst) {
  extern __shared__ __align__(16) unsigned char lds[];
  constexpr int kFragBytes = NT * NT * 1024;
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

  {  // stage the instance: J fragments and h
    const uint4* src = reinterpret_cast<const uint4*>(a.jfrag + (size_t)inst * kFragBytes);
    uint4* dst = reinterpret_cast<uint4*>(lds);
    for (int i = threadIdx.x; i < kFragBytes / 16; i += blockDim.x) dst[i] = src[i];
    if (HAS_H) {
      int32_t* sh = reinterpret_cast<int32_t*>(lds + kFragBytes);
      for (int i = threadIdx.x; i < kNpad; i += blockDim.x) sh[i] = a.h[(size_t)inst * kNpad + i];
    }
  }
  const v4i* sJ = reinterpret_cast<const v4i*>(lds);
  const int32_t* sH = reinterpret_cast<const int32_t*>(lds + kFragBytes);
  int16_t* sTab = reinterpret_cast<int16_t*>(lds + kFragBytes + kHBytes + wave * kTabBytes);
  uint4* sTab4 = reinterpret_cast<uint4*>(sTab);
  __syncthreads();  // the only workgroup barrier

  const int tbase = (tblk * (int)(blockDim.x >> 6) + wave) * 32 * CB;
  if (tbase >= a.R) return;
  int trial[CB];
  bool live[CB];
  size_t cell[CB];
#pragma unroll
  for (int c = 0; c < CB; ++c) {
    trial[c] = tbase + 32 * c + col;
    live[c] = trial[c] < a.R;
    cell[c] = (size_t)inst * a.R + trial[c];
  }
  const uint32_t stream = a.inst_stream[inst];
  const int cls = a.inst_class[inst];
  const uint4* gTab4 = reinterpret_cast<const uint4*>(a.thtab + (size_t)cls * a.T * kTabEntries);
  const int32_t target = a.target ? a.target[inst] : INT_MIN;
  const uint32_t k0 = a.k0, k1 = a.k1;

  // ---- s(0) ----
  v4i B[CB][NT];
#pragma unroll
  for (int c = 0; c < CB; ++c)
#pragma unroll
    for (int mt = 0; mt < NT; ++mt) {
      if (a.init) {
        if (live[c]) B[c][mt] = *reinterpret_cast<const v4i*>(a.init + cell[c] * kNpad + 32 * mt + 16 * half);
        else B[c][mt] = v4i{0x01010101, 0x01010101, 0x01010101, 0x01010101};
      } else {
        const Ctr4 x = philox4x32_10(Ctr4{(uint32_t)(2 * mt + half), 0u, (uint32_t)trial[c],
                                          (kDomainInit << 24) | stream}, k0, k1);
        B[c][mt] = v4i{spins_from_bits(x.x), spins_from_bits(x.y), spins_from_bits(x.z), spins_from_bits(x.w)};
      }
    }

  int32_t e_best[CB], t_best[CB], first_hit[CB], e_cur[CB];
  // noise block of the next row tile, carried across steps (tile 0 of step 0
  // is drawn here so the step loop has no branch after its MFMA chains)
  Ctr4 x_next[CB];
#pragma unroll
  for (int c = 0; c < CB; ++c) {
    e_best[c] = INT_MAX;
    t_best[c] = -1;
    first_hit[c] = -1;
    e_cur[c] = 0;
    x_next[c] = noise_block((uint32_t)half, a.start_step, (uint32_t)trial[c], stream, k0, k1);
  }
  int done = a.T;
  sTab4[lane] = gTab4[lane];  // table of step 0 into buffer 0

  for (int t = 0;; ++t) {
    const int tg = a.start_step + t;
    // Eq. (2) and Eq. (4), one row tile at a time and software-pipelined: the
    // MFMA chains of tile mt+1 (I = J' s over all K tiles) are issued before
    // the VALU work of tile mt, so the matrix core runs while the lanes decide
    // the previous tile's spins.  Per tile: energy of s(t) (Eq. (1),
    // E = -1/2 sum_i s_i (I_i + h_i)) and the update to s(t+1) into Bn; B
    // keeps s(t) until the best-state bookkeeping is done.  At t = T only the
    // energy is used (the update there reads a stale, in-bounds table and is
    // discarded).
    int32_t ep[CB];
    v4i Bn[CB][NT];
    const bool last = (t == a.T);
    const bool has_next = t + 1 < a.T;
    // next step's table (clamped index: a branch-free, always in-bounds load)
    const uint4 nxt = gTab4[(size_t)min(t + 1, a.T - 1) * 64 + lane];
    // centre of this step's table: entry idx in [-256, 256) holds the field
    // threshold for (u, s) with idx = u ^ s (s = +1 -> u ^ 1, s = -1 -> ~u)
    const int16_t* tab = sTab + kNoiseVals;
    uint32_t ctr_trial[CB];
    uint32_t ctr_half = (uint32_t)half;
    PIM_FENCE(ctr_half);
#pragma unroll
    for (int c = 0; c < CB; ++c) {
      ep[c] = 0;
      ctr_trial[c] = (uint32_t)trial[c];
      PIM_FENCE(ctr_trial[c]);
    }
    const v4i* sJl0 = sJ + lane;
    v16i acc_next[CB];
    mfma_row_tile<NT, CB>(sJl0, 0, B, acc_next);
#pragma unroll
    for (int mt = 0; mt < NT; ++mt) {
      v16i acc[CB];
      uint32_t xw[CB][4], bw[CB][4];
#pragma unroll
      for (int c = 0; c < CB; ++c) {
        acc[c] = acc_next[c];
        xw[c][0] = x_next[c].x; xw[c][1] = x_next[c].y; xw[c][2] = x_next[c].z; xw[c][3] = x_next[c].w;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          bw[c][q] = (uint32_t)B[c][mt][q];
          PIM_FENCE(xw[c][q]);
        }
      }
      // fence an integer lane offset, not the pointer: a pointer through the
      // asm would lose its LDS address space and turn the reads into flat loads
      int lane_off = lane;
      PIM_FENCE(lane_off);
      // h of this tile re-read from LDS each step (fenced offset: not hoisted
      // into NT*16 loop-carried registers)
      int hoff = 32 * mt + 16 * half;
      if (HAS_H) PIM_FENCE(hoff);
      const v4i* sJl = sJ + lane_off;
      // (1) LDS: the field thresholds of this tile, indexed by u ^ s
      // registers of this tile that carry decisions (all but the last tile: 16)
      const int kRegs = (mt == NT - 1) ? TAIL : 16;  // a constant once mt is unrolled
      int th[CB][16];
#pragma unroll
      for (int c = 0; c < CB; ++c)
#pragma unroll
        for (int r = 0; r < kRegs; ++r) {
          const int sv = (int)(int8_t)(bw[c][r >> 2] >> (8 * (r & 3)));
          const int idx = (int)((xw[c][r >> 2] >> (8 * (r & 3))) & 0xFFu) ^ sv;
          th[c][r] = tab[idx];
        }
      // (2) independent work that covers the LDS latency: the next tile's MFMA
      //     chains and noise blocks (or the first blocks of the next step)
      if (mt + 1 < NT) mfma_row_tile<NT, CB>(sJl, mt + 1, B, acc_next);
#pragma unroll
      for (int c = 0; c < CB; ++c) {
        if (mt + 1 < NT) x_next[c] = noise_block(2u * (mt + 1) + ctr_half, tg, ctr_trial[c], stream, k0, k1);
        else x_next[c] = noise_block(ctr_half, tg + 1, ctr_trial[c], stream, k0, k1);
      }
      // (3) energy of s(t) and the decisions of this tile
#pragma unroll
      for (int c = 0; c < CB; ++c)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          if (4 * q >= kRegs) {  // padding spins only: kept as they are
            Bn[c][mt][q] = B[c][mt][q];
            continue;
          }
          int d[4];
#pragma unroll
          for (int b = 0; b < 4; ++b) {
            const int r = 4 * q + b;
            const int sv = (int)(int8_t)(bw[c][q] >> (8 * b));
            int I = acc[c][r];
            int v;
            if (HAS_H) {
              const int hv = sH[hoff + r];
              I += hv;
              v = I + hv;
            } else {
              v = I;
            }
            ep[c] += __mul24(sv, v);  // |v| < 2^23: one full-rate 24-bit multiply-add
            d[b] = I - th[c][r];      // >= 0  <=>  s(t+1) = +1
          }
          // sign bytes of d (0xFF where negative) via byte-permute sign
          // replication, then | 0x01 gives the int8 spins +1 / -1
          const uint32_t p01 = __builtin_amdgcn_perm((uint32_t)d[1], (uint32_t)d[0], 0x0C0C0B09u);
          const uint32_t p23 = __builtin_amdgcn_perm((uint32_t)d[3], (uint32_t)d[2], 0x0B090C0Cu);
          Bn[c][mt][q] = (int)(p01 | p23 | 0x01010101u);
        }
      // fence the tile's results as well, so its decisions cannot be sunk
      // past the next tiles' MFMA chains (which would keep every tile's
      // accumulator live at once)
#pragma unroll
      for (int c = 0; c < CB; ++c) {
        PIM_FENCE(ep[c]);
#pragma unroll
        for (int q = 0; q < 4; ++q) PIM_FENCE(Bn[c][mt][q]);
      }
      __builtin_amdgcn_sched_barrier(0);
    }
#pragma unroll
    for (int c = 0; c < CB; ++c) {
      if (RECORD && live[c]) {  // diagnostics: keep s(t) of every step
        size_t off = (cell[c] * (size_t)(a.T + 1) + t) * kNpad + 16 * half;
        PIM_FENCE(off);
        int8_t* dst = a.trace + off;
#pragma unroll
        for (int mt = 0; mt < NT; ++mt) *reinterpret_cast<v4i*>(dst + 32 * mt) = B[c][mt];
      }
      const int32_t epc = ep[c] + __shfl_xor(ep[c], 32);
      const int32_t E = -(epc / 2);
      if (E < e_best[c]) {
        e_best[c] = E;
        t_best[c] = tg;
        if (live[c]) {
          // address formed here (opaque base, immediate tile offsets) rather
          // than hoisted per tile out of the step loop
          size_t off = cell[c] * kNpad + 16 * half;
          PIM_FENCE(off);
          int8_t* dst = a.best_s + off;
#pragma unroll
          for (int mt = 0; mt < NT; ++mt) *reinterpret_cast<v4i*>(dst + 32 * mt) = B[c][mt];
        }
      }
      if (first_hit[c] < 0 && E <= target) first_hit[c] = tg;
      e_cur[c] = E;
    }
    if (last) break;
    if ((t & 255) == 0 && __atomic_load_n(a.cancel, __ATOMIC_RELAXED) != 0) {
      done = t;  // s(t) stays the final state
      break;
    }
#pragma unroll
    for (int c = 0; c < CB; ++c)
#pragma unroll
      for (int mt = 0; mt < NT; ++mt) B[c][mt] = Bn[c][mt];
    if (has_next) {
      // every lookup of this step precedes this write in the wave's LDS order
      sTab4[lane] = nxt;
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
  }

#pragma unroll
  for (int c = 0; c < CB; ++c) {
    if (!live[c]) continue;
#pragma unroll
    for (int mt = 0; mt < NT; ++mt)
      *reinterpret_cast<v4i*>(a.final_s + cell[c] * kNpad + 32 * mt + 16 * half) = B[c][mt];
    if (half == 0) {
      a.e_best[cell[c]] = e_best[c];
      a.t_best[cell[c]] = t_best[c];
      a.first_hit[cell[c]] = first_hit[c];
      a.e_final[cell[c]] = e_cur[c];
      a.steps_done[cell[c]] = done;
    }
  }
}

constexpr int kBlocksPerWave = 1;  // CB: 32-trial column blocks per wave

template <int NT, bool HAS_H, bool RECORD, int TAIL>
hipError_t launch_tail(const SweepArgs& a, int count, hipStream_t s) {
  const int waves = a.waves;  // 1, 2 or 4 (checked by the caller)
  const size_t lds = (size_t)NT * NT * 1024 + (HAS_H ? NT * 32 * 4 : 0) + (size_t)waves * kTabBytes;
  auto kern = sweep_mfma_kernel<NT, kBlocksPerWave, HAS_H, RECORD, TAIL>;
  hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  const int per_wg = 32 * kBlocksPerWave * waves;
  const int bpi = (a.R + per_wg - 1) / per_wg;
  const int groups = (count + kXcds - 1) / kXcds;
  const dim3 grid((unsigned)(bpi * groups * kXcds));
  hipLaunchKernelGGL(kern, grid, dim3(64 * waves), lds, s, a, bpi);
  return hipGetLastError();
}

// registers of the last row tile that carry spins below N (in the lower lane
// half), rounded up to 4; recording runs always take the full tile
template <int NT, bool HAS_H, bool RECORD>
hipError_t launch_nt(const SweepArgs& a, int count, hipStream_t s) {
  const int rem = a.n - 32 * (NT - 1);  // 1 .. 32
  if (RECORD || rem > 12) return launch_tail<NT, HAS_H, RECORD, 16>(a, count, s);
  if (rem > 8) return launch_tail<NT, HAS_H, RECORD, 12>(a, count, s);
  if (rem > 4) return launch_tail<NT, HAS_H, RECORD, 8>(a, count, s);
  return launch_tail<NT, HAS_H, RECORD, 4>(a, count, s);
}

template <bool HAS_H, bool RECORD>
hipError_t launch_h(const SweepArgs& a, int count, int nt, hipStream_t s) {
  switch (nt) {
    case 1: return launch_nt<1, HAS_H, RECORD>(a, count, s);
    case 2: return launch_nt<2, HAS_H, RECORD>(a, count, s);
    case 3: return launch_nt<3, HAS_H, RECORD>(a, count, s);
    case 4: return launch_nt<4, HAS_H, RECORD>(a, count, s);
    case 5: return launch_nt<5, HAS_H, RECORD>(a, count, s);
    case 6: return launch_nt<6, HAS_H, RECORD>(a, count, s);
    case 7: return launch_nt<7, HAS_H, RECORD>(a, count, s);
    case 8: return launch_nt<8, HAS_H, RECORD>(a, count, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace

hipError_t launch_sweep_mfma(const SweepArgs& a, int count, int nt, bool has_h, hipStream_t s) {
  if (a.npad != nt * 32) return hipErrorInvalidValue;
  if (a.waves != 1 && a.waves != 2 && a.waves != kWaves) return hipErrorInvalidValue;
  if (a.trace) return has_h ? launch_h<true, true>(a, count, nt, s) : launch_h<false, true>(a, count, nt, s);
  return has_h ? launch_h<true, false>(a, count, nt, s) : launch_h<false, false>(a, count, nt, s);
}

void pack_mfma_fragments(const int8_t* J, int n, int nt, int8_t* out) {
  for (int mt = 0; mt < nt; ++mt)
    for (int kt = 0; kt < nt; ++kt)
      for (int l = 0; l < 64; ++l) {
        const int m = l & 31, hh = l >> 5;
        // physical output row m of tile mt carries spin 32mt + 16*((m/4)%2) + 4*(m/8) + m%4
        const int row = 32 * mt + 16 * ((m >> 2) & 1) + 4 * (m >> 3) + (m & 3);
        for (int p = 0; p < 16; ++p) {
          const int colj = 32 * kt + 16 * hh + p;  // K-slot (hh, p) carries spin 32kt + 16hh + p
          const int8_t v = (row < n && colj < n) ? J[(size_t)row * n + colj] : (int8_t)0;
          out[(((size_t)mt * nt + kt) * 64 + l) * 16 + p] = v;
        }
      }
}

}  // namespace pim
