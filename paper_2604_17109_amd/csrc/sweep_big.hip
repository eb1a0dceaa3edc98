// PIMI sweep on int8 MFMA for 256 < N <= 1024, where N^2 bytes of couplings no
// longer fit in LDS and the step is a true dense contraction
// I[N x R] = J[N x N] . S[N x R] (Eq. (2)) that has to stream J.
//
// One workgroup = 8 waves (two per SIMD) on 128 trials (four 32-trial column
// blocks) of one instance.  The waves split the row tiles: wave w owns row
// tiles mt = w, w + 8, w + 16, w + 24.  For a row tile the wave runs the
// contraction of all four column blocks at once: every A fragment of J (read
// from global memory, i.e. L2 / the last-level cache) feeds four
// v_mfma_i32_32x32x32_i8, so J is read once per workgroup and step for 128
// trials.  The B operand, the spins s(t) of the 128 trials, lives in one LDS
// buffer that every wave reads.
//
// A step runs in two phases separated by workgroup barriers:
//   1. contraction and decisions (Eq. (4)) of the wave's row tiles; the new
//      spins s(t+1) stay in registers, the per-trial partial energies
//      (Eq. (1)) go to LDS;
//   -- barrier: every wave has finished reading s(t) --
//   2. energies of s(t) reduced over the waves, best-state bookkeeping (s(t)
//      is still in LDS), then s(t+1) and the next step's threshold table are
//      written in place;
//   -- barrier: s(t+1) is complete --
//
// Workgroups are mapped so that all blocks of one instance run on one XCD
// (hardware dispatch sends consecutive workgroups to consecutive XCDs), which
// keeps the instance's couplings in that XCD's L2.
#include <hip/hip_runtime.h>

#include <climits>
#include <cstdint>

#include "internal.hpp"
#include "philox.hpp"
#include "frag_stream.hpp"

namespace pim {
namespace {

typedef int v4i __attribute__((ext_vector_type(4)));
typedef int v16i __attribute__((ext_vector_type(16)));

constexpr int kWaves = 8;            // two waves per SIMD
constexpr int kCB = 4;               // 32-trial column blocks per workgroup
constexpr int kTrialsWG = 32 * kCB;  // trials per workgroup
constexpr int kXcds = 8;
constexpr int kTabBytes = kTabEntries * 2;
constexpr int kMinTiles = PIM_MAX_N_LDS / 32 + 1;  // 9
constexpr int kMaxTiles = PIM_MAX_N / 32;          // 32

#define PIM_FENCE(v) asm volatile("" : "+v"(v))

__device__ __forceinline__ int spins_from_bits(uint32_t w) {
  return (int)(0xFFFFFFFFu - 0xFEu * ((w >> 7) & 0x01010101u));
}

__device__ __forceinline__ Ctr4 noise_block(uint32_t block, int tg, uint32_t trial, uint32_t stream,
                                            uint32_t k0, uint32_t k1) {
  return philox4x32_10(Ctr4{block, (uint32_t)tg, trial, (kDomainNoise << 24) | stream}, k0, k1);
}

// Workgroup barrier for data exchanged through LDS only: each wave waits for
// its own LDS operations, not for its outstanding global loads (prefetches
// stay in flight across it).  A plain __syncthreads() is also a fence for
// global memory and would drain every prefetch at every step.
__device__ __forceinline__ void lds_barrier() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// LDS spin buffer: tile kt of column block c, lane l at ((kt * kCB + c) * 64 + l).
__device__ __forceinline__ int sb_index(int kt, int c, int lane) { return (kt * kCB + c) * 64 + lane; }

// Fields of MT (1 or 2) row tiles mt0, mt0 + kWaves for the four column
// blocks: nt K steps, each MT A fragments from global memory and four B
// fragments from LDS, MT x 4 MFMAs.  With two row tiles every B fragment read
// from LDS feeds two MFMAs, which halves the LDS traffic per MFMA and doubles
// the matrix work that covers each LDS read.
//
// The A fragments stream through a register ring of D slots per row tile (K
// step kt uses slot kt % D and, right after its MFMAs are issued, refills
// that slot with the fragment D K steps ahead, from a clamped, always
// in-bounds index); the B fragments of the next K step are read into the
// same registers right after the MFMAs that consume them are issued.  The K
// steps run in unconditional groups of D followed by a tail of fewer than D;
// a scheduling barrier per K step keeps the compiler from hoisting more
// operand loads than these registers.  Fragment indices are wave-uniform
// (scalar) and the lane offset is a 32-bit register: each load is a scalar
// base plus one 32-bit vector offset.  K step 0 is peeled so its MFMAs take a
// zero accumulator as an inline constant (inside the loop the accumulators
// would have to be zeroed by moves, one per register); K step k uses ring
// slot k % D.
template <int MT>
__device__ __forceinline__ void big_rows(const FragStream& gA, const v4i* sB, int lane, int mt0, int nt,
                                         v16i (&acc)[MT][kCB]) {
  constexpr int D = MT == 1 ? 4 : 2;
  int fa[MT];
#pragma unroll
  for (int r = 0; r < MT; ++r) fa[r] = (mt0 + kWaves * r) * nt;
  v4i ar[MT][D], b[kCB];
#pragma unroll
  for (int r = 0; r < MT; ++r)
#pragma unroll
    for (int i = 0; i < D; ++i) ar[r][i] = gA(fa[r] + i);  // nt >= 9 > D
#pragma unroll
  for (int c = 0; c < kCB; ++c) b[c] = sB[sb_index(0, c, lane)];
  // K step 0
#pragma unroll
  for (int c = 0; c < kCB; ++c)
#pragma unroll
    for (int r = 0; r < MT; ++r) acc[r][c] = __builtin_amdgcn_mfma_i32_32x32x32_i8(ar[r][0], b[c], v16i{}, 0, 0, 0);
#pragma unroll
  for (int r = 0; r < MT; ++r) ar[r][0] = gA(fa[r] + D);  // D < nt
#pragma unroll
  for (int c = 0; c < kCB; ++c) b[c] = sB[sb_index(1, c, lane)];
  __builtin_amdgcn_sched_barrier(0);
  // K steps 1 .. nt - 1: groups of D (K step kt + i, kt = 1 mod D, in slot
  // (1 + i) % D), then a tail of fewer than D
  const int nfull = 1 + (nt - 1) - (nt - 1) % D;
  int kt = 1;
  for (; kt < nfull; kt += D) {
#pragma unroll
    for (int i = 0; i < D; ++i) {
      const int slot = (1 + i) % D;
#pragma unroll
      for (int c = 0; c < kCB; ++c)
#pragma unroll
        for (int r = 0; r < MT; ++r)
          acc[r][c] = __builtin_amdgcn_mfma_i32_32x32x32_i8(ar[r][slot], b[c], acc[r][c], 0, 0, 0);
      // refill the slot after its last use, so the load lands in place
      const int kf = min(kt + i + D, nt - 1);
#pragma unroll
      for (int r = 0; r < MT; ++r) ar[r][slot] = gA(fa[r] + kf);
      const int kn = min(kt + i + 1, nt - 1);
#pragma unroll
      for (int c = 0; c < kCB; ++c) b[c] = sB[sb_index(kn, c, lane)];
      __builtin_amdgcn_sched_barrier(0);
    }
  }
#pragma unroll
  for (int i = 0; i < D - 1; ++i) {
    if (kt + i < nt) {  // uniform
      const int slot = (1 + i) % D;
#pragma unroll
      for (int c = 0; c < kCB; ++c)
#pragma unroll
        for (int r = 0; r < MT; ++r)
          acc[r][c] = __builtin_amdgcn_mfma_i32_32x32x32_i8(ar[r][slot], b[c], acc[r][c], 0, 0, 0);
      if (kt + i + 1 < nt) {
#pragma unroll
        for (int c = 0; c < kCB; ++c) b[c] = sB[sb_index(kt + i + 1, c, lane)];
      }
    }
  }
}

// Eq. (4) decisions and the Eq. (1) energy terms of row tile mt for the four
// column blocks, one block at a time: s(t+1) of the tile into bn, the partial
// sums s_i (I_i + h_i) into ep.
template <bool HAS_H>
__device__ __forceinline__ void big_decide(const v16i (&acc)[kCB], const v4i* sB, const int32_t* sH,
                                           const int16_t* tab, int mt, int lane_off, int half, uint32_t ctr_half,
                                           uint32_t ctr_trial, int tg, uint32_t stream, uint32_t k0, uint32_t k1,
                                           v4i (&bn)[kCB], int32_t (&ep)[kCB]) {
  const int hoff = 32 * mt + 16 * half;
#pragma unroll
  for (int c = 0; c < kCB; ++c) {
    const Ctr4 x = noise_block(2u * mt + ctr_half, tg, ctr_trial + 32u * c, stream, k0, k1);
    uint32_t xw[4] = {x.x, x.y, x.z, x.w};
    const v4i cv = sB[sb_index(mt, c, lane_off)];
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
    // h of this row tile re-read for every column block (fenced offset)
    int hoff_c = hoff;
    if (HAS_H) PIM_FENCE(hoff_c);
    v4i o;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      int d[4];
#pragma unroll
      for (int bb = 0; bb < 4; ++bb) {
        const int r = 4 * q + bb;
        const int sv = (int)(int8_t)(bw[q] >> (8 * bb));
        int I = acc[c][r];
        int v = I;
        if (HAS_H) {
          const int hv = sH[hoff_c + r];
          I += hv;
          v = I + hv;
        }
        ep[c] += __mul24(sv, v);  // |v| < 2^23
        d[bb] = I - th[r];        // >= 0  <=>  s(t+1) = +1
      }
      // sign bytes of d via byte-permute sign replication, | 0x01 -> +1 / -1
      const uint32_t p01 = __builtin_amdgcn_perm((uint32_t)d[1], (uint32_t)d[0], 0x0C0C0B09u);
      const uint32_t p23 = __builtin_amdgcn_perm((uint32_t)d[3], (uint32_t)d[2], 0x0B090C0Cu);
      o[q] = (int)(p01 | p23 | 0x01010101u);
    }
    bn[c] = o;
    PIM_FENCE(ep[c]);
#pragma unroll
    for (int q = 0; q < 4; ++q) PIM_FENCE(bn[c][q]);
    // one column block's decisions at a time (bounds the live temporaries)
    __builtin_amdgcn_sched_barrier(0);
  }
}

// One workgroup's run: trial block tblk (128 trials) of instance inst.
template <int RPW, bool HAS_H>
__device__ __forceinline__ void big_body(const SweepArgs& a, int nt, int inst, int tblk) {
  extern __shared__ __align__(16) unsigned char lds[];
  const int npad = nt * 32;
  // LDS: spins [nt][kCB][64] x 16 B | table 1 KB | energy partials
  // [kWaves][kCB][32] | per-trial t_best, first_hit, e_cur [3][kCB][32] |
  // cancel flag | h
  v4i* sB = reinterpret_cast<v4i*>(lds);
  int16_t* sTab = reinterpret_cast<int16_t*>(lds + (size_t)nt * kCB * 1024);
  int32_t* sE = reinterpret_cast<int32_t*>(lds + (size_t)nt * kCB * 1024 + kTabBytes);
  int32_t* sStat = sE + kWaves * kCB * 32;
  int32_t* sFlag = sStat + 3 * kCB * 32;
  int32_t* sH = sFlag + 4;

  // wave index made scalar: every row-tile index below is wave-uniform
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  const int col = lane & 31;
  const int half = lane >> 5;
  // trial of column block c: trial0 + 32 c (recomputed where used, which
  // keeps the per-lane bookkeeping out of the register budget)
  const int trial0 = tblk * kTrialsWG + col;
  const size_t cell0 = (size_t)inst * a.R + trial0;
  // the writer of the per-trial statistics: one lane per trial
  const bool writer = wave == 0 && half == 0;
  const uint32_t stream = a.inst_stream[inst];
  const int cls = a.inst_class[inst];
  const uint4* gTab4 = reinterpret_cast<const uint4*>(a.thtab + (size_t)cls * a.T * kTabEntries);
  const int32_t target = a.target ? a.target[inst] : INT_MIN;
  const uint32_t k0 = a.k0, k1 = a.k1;
  // the instance's A fragments (fragment mt * nt + p; at most 32 * 32 of 1 KB)
  const FragStream gA(a.jfrag + (size_t)inst * nt * nt * 1024, (uint32_t)(nt * nt * 1024), lane);

  if (HAS_H)
    for (int i = threadIdx.x; i < npad; i += 64 * kWaves) sH[i] = a.h[(size_t)inst * npad + i];
  // s(0): each wave its own row tiles
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
        v = v4i{spins_from_bits(x.x), spins_from_bits(x.y), spins_from_bits(x.z), spins_from_bits(x.w)};
      }
      sB[sb_index(mt, c, lane)] = v;
    }
  }
  if (wave == 0) reinterpret_cast<uint4*>(sTab)[lane] = gTab4[lane];
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
  // row tiles of this wave: wave + kWaves j for j < rw (rw >= 1: nt >= 9 > wave)
  const int rw = (nt - wave + kWaves - 1) / kWaves;
  // centre of the step table: entry idx in [-256, 256) holds the field
  // threshold for (u, s) with idx = u ^ s (s = +1 -> u ^ 1, s = -1 -> ~u)
  const int16_t* tab = sTab + kNoiseVals;
  for (int t = 0;; ++t) {
    const int tg = a.start_step + t;
    // wave 0 fetches the table of step t+1 (written after the first barrier)
    uint4 nxt = uint4{0, 0, 0, 0};
    if (wave == 0) nxt = gTab4[(size_t)min(t + 1, a.T - 1) * 64 + lane];
    int32_t ep[kCB];
    v4i Bn[RPW][kCB];
#pragma unroll
    for (int c = 0; c < kCB; ++c) ep[c] = 0;
    // counter words and lane offsets re-materialised each step through
    // fences: otherwise the loop-invariant parts of every (row tile, column
    // block) noise block and LDS address are hoisted out of the step loop
    // into registers this kernel does not have
    uint32_t ctr_half = (uint32_t)half, ctr_trial = (uint32_t)trial0;
    int lane_off = lane;
    PIM_FENCE(ctr_half);
    PIM_FENCE(ctr_trial);
    PIM_FENCE(lane_off);
    // ---- phase 1: contraction and decisions of the wave's row tiles ----
    // row tiles mt = wave + kWaves j, j < rw, taken in pairs (j, j + 1); an
    // odd last one alone
#pragma unroll
    for (int g = 0; g < (RPW + 1) / 2; ++g) {
      const int j0 = 2 * g;
      if (j0 >= rw) break;  // uniform
      const int mt0 = wave + kWaves * j0;
      if (j0 + 1 < rw) {
        v16i acc[2][kCB];
        big_rows<2>(gA, sB, lane_off, mt0, nt, acc);
        big_decide<HAS_H>(acc[0], sB, sH, tab, mt0, lane_off, half, ctr_half, ctr_trial, tg, stream, k0, k1,
                          Bn[j0], ep);
        if (j0 + 1 < RPW)
          big_decide<HAS_H>(acc[1], sB, sH, tab, mt0 + kWaves, lane_off, half, ctr_half, ctr_trial, tg, stream,
                            k0, k1, Bn[j0 + 1 < RPW ? j0 + 1 : j0], ep);
      } else {
        v16i acc[1][kCB];
        big_rows<1>(gA, sB, lane_off, mt0, nt, acc);
        big_decide<HAS_H>(acc[0], sB, sH, tab, mt0, lane_off, half, ctr_half, ctr_trial, tg, stream, k0, k1,
                          Bn[j0], ep);
      }
    }
    // per-trial partial energies of this wave's rows (both lane halves)
#pragma unroll
    for (int c = 0; c < kCB; ++c) {
      const int32_t epc = ep[c] + __shfl_xor(ep[c], 32);
      if (half == 0) sE[(wave * kCB + c) * 32 + col] = epc;
    }
    if (threadIdx.x == 0 && (t & 255) == 0 && t < a.T)
      sFlag[0] = __atomic_load_n(a.cancel, __ATOMIC_RELAXED) != 0 ? 1 : 0;
    lds_barrier();  // every read of s(t) and of the table is done; energies of s(t) complete
    // ---- phase 2: energies, bookkeeping, s(t+1) in place ----
#pragma unroll
    for (int c = 0; c < kCB; ++c) {
      int32_t tot = 0;
#pragma unroll
      for (int w = 0; w < kWaves; ++w) tot += sE[(w * kCB + c) * 32 + col];
      const int32_t E = -(tot / 2);
      if (E < e_best[c]) {
        e_best[c] = E;
        if (writer) sStat[(0 * kCB + c) * 32 + col] = tg;
        if ((trial0 + 32 * c < a.R)) {
          // address formed here from a fenced offset (not hoisted out of the
          // step loop into registers for every column block)
          size_t off = (cell0 + 32 * c) * npad + 16 * half;
          PIM_FENCE(off);
          int8_t* dst = a.best_s + off;
#pragma unroll
          for (int j = 0; j < RPW; ++j) {
            const int mt = wave + kWaves * j;
            if (mt < nt) *reinterpret_cast<v4i*>(dst + 32 * mt) = sB[sb_index(mt, c, lane)];
          }
        }
      }
      if (writer) {
        if (sStat[(1 * kCB + c) * 32 + col] < 0 && E <= target) sStat[(1 * kCB + c) * 32 + col] = tg;
        sStat[(2 * kCB + c) * 32 + col] = E;
      }
    }
    if (t == a.T) break;  // uniform: s(T) stays in LDS
    const bool stop = (t & 255) == 0 && sFlag[0] != 0;  // uniform: written before the barrier
    if (stop) {
      done = t;  // s(t) stays the final state
      break;
    }
#pragma unroll
    for (int j = 0; j < RPW; ++j) {
      const int mt = wave + kWaves * j;
      if (mt >= nt) break;
#pragma unroll
      for (int c = 0; c < kCB; ++c) sB[sb_index(mt, c, lane)] = Bn[j][c];
    }
    if (wave == 0) reinterpret_cast<uint4*>(sTab)[lane] = nxt;
    lds_barrier();  // s(t+1) and the table of step t+1 are complete
  }
  // final state: the s(t) left in LDS
#pragma unroll
  for (int c = 0; c < kCB; ++c) {
    if (!(trial0 + 32 * c < a.R)) continue;
#pragma unroll
    for (int j = 0; j < RPW; ++j) {
      const int mt = wave + kWaves * j;
      if (mt < nt)
        *reinterpret_cast<v4i*>(a.final_s + (cell0 + 32 * c) * npad + 32 * mt + 16 * half) = sB[sb_index(mt, c, lane)];
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
__global__ __launch_bounds__(64 * kWaves, 2) void sweep_big_kernel(SweepArgs a, int nt, int blocks_per_inst) {
  // workgroup -> (instance, trial block): the blocks of instance k all have
  // linear ids congruent to k modulo the XCD count (hardware dispatch sends
  // consecutive workgroups to consecutive XCDs), so they share one L2
  const int lin = blockIdx.x;
  const int inst = (lin % kXcds) + kXcds * ((lin / kXcds) / blocks_per_inst);
  const int tblk = (lin / kXcds) % blocks_per_inst;
  if (inst >= a.count) return;  // whole workgroup: before any barrier
  big_body<RPW, HAS_H>(a, nt, inst, tblk);
}

// Several batches of different N in one launch: workgroup b runs work item
// work[b] = (part, instance, trial block) with that part's arguments.  The
// host orders the items so that workgroups 8k + x all run on XCD x, each
// instance's blocks on one XCD, and each XCD's items longest first.
template <bool HAS_H>
__global__ __launch_bounds__(64 * kWaves, 2) void sweep_big_multi_kernel(const MultiPart* parts, const int4* work,
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
  big_body<kMaxTiles / kWaves, HAS_H>(a, nt, item.y, item.z);
}

size_t big_lds_bytes(int nt, bool has_h) {
  return (size_t)nt * kCB * 1024 + kTabBytes + (size_t)(kWaves + 3) * kCB * 32 * 4 + 16 +
         (has_h ? (size_t)nt * 32 * 4 : 0);
}

template <int RPW, bool HAS_H>
hipError_t launch_rpw(const SweepArgs& a, int count, int nt, hipStream_t s) {
  const size_t lds = big_lds_bytes(nt, HAS_H);
  auto kern = sweep_big_kernel<RPW, HAS_H>;
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
hipError_t launch_multi(const MultiPart* d_parts, const int4* d_work, int nwork, int nt_max, const MultiRun& run,
                        hipStream_t s) {
  const size_t lds = big_lds_bytes(nt_max, HAS_H);
  auto kern = sweep_big_multi_kernel<HAS_H>;
  hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(kern), hipFuncAttributeMaxDynamicSharedMemorySize,
                                     (int)lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(kern, dim3((unsigned)nwork), dim3(64 * kWaves), lds, s, d_parts, d_work, nwork, run);
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

}  // namespace

int big_tiles(int n) { return (n + 31) / 32; }

hipError_t launch_sweep_big_multi(const MultiPart* d_parts, const int4* d_work, int nwork, int nt_max, bool has_h,
                                  const MultiRun& run, hipStream_t s) {
  if (nwork < 1 || nt_max < kMinTiles || nt_max > kMaxTiles) return hipErrorInvalidValue;
  return has_h ? launch_multi<true>(d_parts, d_work, nwork, nt_max, run, s)
               : launch_multi<false>(d_parts, d_work, nwork, nt_max, run, s);
}

// Relative time of one workgroup-step at nt row tiles, the form of the e2m1
// kernel's model with int8 K steps of 32 (nt per tile instead of nt / 2):
// the waves of a SIMD (w and w + 4) run their tiles' contractions and
// decisions one after the other, and the workgroup waits at every step for
// its busiest SIMD.
double big_step_cost(int nt) {
  int simd_tiles = 0;
  for (int w = 0; w < kWaves / 2; ++w) {
    const int t = (nt - w + kWaves - 1) / kWaves + (nt - w - kWaves / 2 + kWaves - 1) / kWaves;
    simd_tiles = t > simd_tiles ? t : simd_tiles;
  }
  return simd_tiles * (128.0 * nt + 2660.0) + 3000.0;
}

hipError_t launch_sweep_big(const SweepArgs& a, int count, int nt, bool has_h, hipStream_t s) {
  if (a.npad != nt * 32 || nt < kMinTiles || nt > kMaxTiles || a.T < 1 || count < 1 || a.R < 1)
    return hipErrorInvalidValue;
  return has_h ? launch_h<true>(a, count, nt, s) : launch_h<false>(a, count, nt, s);
}

}  // namespace pim
