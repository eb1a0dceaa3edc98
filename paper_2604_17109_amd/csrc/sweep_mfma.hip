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
// Each wave double-buffers that 1 KB table in LDS and streams the next step's
// copy from global memory while it works on the current one.
#include <hip/hip_runtime.h>

#include <climits>
#include <cstdint>

#include "internal.hpp"
#include "philox.hpp"

namespace pim {
namespace {

typedef int v4i __attribute__((ext_vector_type(4)));
typedef int v16i __attribute__((ext_vector_type(16)));

constexpr int kWaves = 4;                 // waves (32-trial blocks) per workgroup
constexpr int kTabBytes = kTabEntries * 2;  // 1 KB per step table
static_assert(kTabBytes == 64 * 16, "one 16-byte chunk per lane");

// +1 where the byte's top bit (u >= 128) is set, -1 elsewhere.
__device__ __forceinline__ int spins_from_bits(uint32_t w) {
  return (int)(0xFFFFFFFFu - 0xFEu * ((w >> 7) & 0x01010101u));
}

template <int NT, bool HAS_H>
__global__ __launch_bounds__(64 * kWaves, (NT <= 4 ? 2 : 1)) void sweep_mfma_kernel(SweepArgs a) {
  extern __shared__ __align__(16) unsigned char lds[];
  constexpr int kFragBytes = NT * NT * 1024;
  constexpr int kNpad = NT * 32;
  constexpr int kHBytes = HAS_H ? kNpad * 4 : 0;
  const int inst = blockIdx.y;
  const int wave = threadIdx.x >> 6;
  const int lane = threadIdx.x & 63;
  const int col = lane & 31;
  const int half = lane >> 5;

  {  // stage the instance: J fragments and h
    const uint4* src = reinterpret_cast<const uint4*>(a.jfrag + (size_t)inst * kFragBytes);
    uint4* dst = reinterpret_cast<uint4*>(lds);
    for (int i = threadIdx.x; i < kFragBytes / 16; i += 64 * kWaves) dst[i] = src[i];
    if (HAS_H) {
      int32_t* sh = reinterpret_cast<int32_t*>(lds + kFragBytes);
      for (int i = threadIdx.x; i < kNpad; i += 64 * kWaves) sh[i] = a.h[(size_t)inst * kNpad + i];
    }
  }
  const v4i* sJ = reinterpret_cast<const v4i*>(lds);
  // volatile: re-read h each step instead of pinning NT*16 registers for it
  const volatile int32_t* sH = reinterpret_cast<const volatile int32_t*>(lds + kFragBytes);
  int16_t* sTab = reinterpret_cast<int16_t*>(lds + kFragBytes + kHBytes + wave * 2 * kTabBytes);
  uint4* sTab4 = reinterpret_cast<uint4*>(sTab);
  __syncthreads();  // the only workgroup barrier

  const int wblock = blockIdx.x * kWaves + wave;
  if (wblock * 32 >= a.R) return;
  const int trial = wblock * 32 + col;
  const bool live = trial < a.R;
  const size_t cell = (size_t)inst * a.R + trial;
  const uint32_t stream = a.inst_stream[inst];
  const int cls = a.inst_class[inst];
  const uint4* gTab4 = reinterpret_cast<const uint4*>(a.thtab + (size_t)cls * a.T * kTabEntries);
  const int32_t target = a.target ? a.target[inst] : INT_MIN;
  const uint32_t k0 = a.k0, k1 = a.k1;

  // ---- s(0) ----
  v4i B[NT];
#pragma unroll
  for (int mt = 0; mt < NT; ++mt) {
    if (a.init) {
      if (live) B[mt] = *reinterpret_cast<const v4i*>(a.init + cell * kNpad + 32 * mt + 16 * half);
      else B[mt] = v4i{0x01010101, 0x01010101, 0x01010101, 0x01010101};
    } else {
      const Ctr4 x = philox4x32_10(Ctr4{(uint32_t)(2 * mt + half), 0u, (uint32_t)trial,
                                        (kDomainInit << 24) | stream}, k0, k1);
      B[mt] = v4i{spins_from_bits(x.x), spins_from_bits(x.y), spins_from_bits(x.z), spins_from_bits(x.w)};
    }
  }

  int32_t e_best = INT_MAX, t_best = -1, first_hit = -1, e_cur = 0;
  int done = a.T;
  sTab4[lane] = gTab4[lane];  // table of step 0 into buffer 0

  for (int t = 0;; ++t) {
    const int tg = a.start_step + t;
    // ---- Eq. (2): I = J s (+ h), one MFMA chain per row tile ----
    v16i acc[NT];
#pragma unroll
    for (int mt = 0; mt < NT; ++mt) acc[mt] = v16i{};
#pragma unroll
    for (int kt = 0; kt < NT; ++kt) {
#pragma unroll
      for (int mt = 0; mt < NT; ++mt)
        acc[mt] = __builtin_amdgcn_mfma_i32_32x32x32_i8(sJ[(mt * NT + kt) * 64 + lane], B[kt], acc[mt], 0, 0, 0);
      // keep at most one K tile of A fragments in flight (register pressure)
      __builtin_amdgcn_sched_barrier(0);
    }
    if (HAS_H) {
#pragma unroll
      for (int mt = 0; mt < NT; ++mt)
#pragma unroll
        for (int r = 0; r < 16; ++r) acc[mt][r] += sH[32 * mt + 16 * half + r];
    }
    // One pass over the 16*NT fields of the lane: the energy of s(t) (Eq. (1),
    // E = -1/2 sum_i s_i (I_i + h_i)) and, unless t = T, the update to s(t+1)
    // (Eq. (4)) into Bn.  B keeps s(t) until the best-state bookkeeping is done.
    int32_t ep = 0;
    v4i Bn[NT];
    const bool last = (t == a.T);
    uint4 nxt = uint4{0, 0, 0, 0};
    const bool has_next = t + 1 < a.T;
    if (has_next) nxt = gTab4[(size_t)(t + 1) * 64 + lane];
    if (last) {
#pragma unroll
      for (int mt = 0; mt < NT; ++mt)
#pragma unroll
        for (int r = 0; r < 16; ++r) {
          const int s = (int)(int8_t)((uint32_t)B[mt][r >> 2] >> (8 * (r & 3)));
          int v = acc[mt][r];
          if (HAS_H) v += sH[32 * mt + 16 * half + r];
          ep += __mul24(s, v);
        }
    } else {
      // centre of this step's table: entry idx in [-256, 256) holds the field
      // threshold for (u, s) with idx = u ^ s (s = +1 -> u ^ 1, s = -1 -> ~u)
      const int16_t* tab = sTab + (t & 1) * kTabEntries + kNoiseVals;
#pragma unroll
      for (int mt = 0; mt < NT; ++mt) {
        const Ctr4 x = philox4x32_10(Ctr4{(uint32_t)(2 * mt + half), (uint32_t)tg, (uint32_t)trial,
                                          (kDomainNoise << 24) | stream}, k0, k1);
        const uint32_t xw[4] = {x.x, x.y, x.z, x.w};
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const uint32_t sw = (uint32_t)B[mt][q];
          int d[4];
#pragma unroll
          for (int b = 0; b < 4; ++b) {
            const int s = (int)(int8_t)(sw >> (8 * b));
            const int I = acc[mt][4 * q + b];
            int v = I;
            if (HAS_H) v += sH[32 * mt + 16 * half + 4 * q + b];
            ep += __mul24(s, v);  // |v| < 2^23: one full-rate 24-bit multiply-add
            const int idx = (int)((xw[q] >> (8 * b)) & 0xFFu) ^ s;
            d[b] = I - (int)tab[idx];  // >= 0  <=>  s(t+1) = +1
          }
          // sign bytes of d (0xFF where negative) via byte-permute sign
          // replication, then | 0x01 gives the int8 spins +1 / -1
          const uint32_t p01 = __builtin_amdgcn_perm((uint32_t)d[1], (uint32_t)d[0], 0x0C0C0B09u);
          const uint32_t p23 = __builtin_amdgcn_perm((uint32_t)d[3], (uint32_t)d[2], 0x0B090C0Cu);
          Bn[mt][q] = (int)(p01 | p23 | 0x01010101u);
        }
        // one row tile's lookups in flight at a time (register pressure)
        __builtin_amdgcn_sched_barrier(0);
      }
    }
    ep += __shfl_xor(ep, 32);
    const int32_t E = -(ep / 2);
    if (E < e_best) {
      e_best = E;
      t_best = tg;
      if (live) {
#pragma unroll
        for (int mt = 0; mt < NT; ++mt)
          *reinterpret_cast<v4i*>(a.best_s + cell * kNpad + 32 * mt + 16 * half) = B[mt];
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
    for (int mt = 0; mt < NT; ++mt) B[mt] = Bn[mt];
    if (has_next) {
      sTab4[((t + 1) & 1) * 64 + lane] = nxt;
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
  }

  if (live) {
#pragma unroll
    for (int mt = 0; mt < NT; ++mt)
      *reinterpret_cast<v4i*>(a.final_s + cell * kNpad + 32 * mt + 16 * half) = B[mt];
    if (half == 0) {
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
  const size_t lds = (size_t)NT * NT * 1024 + (HAS_H ? NT * 32 * 4 : 0) + (size_t)kWaves * 2 * kTabBytes;
  auto kern = sweep_mfma_kernel<NT, HAS_H>;
  hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  const dim3 grid((a.R + 32 * kWaves - 1) / (32 * kWaves), count);
  hipLaunchKernelGGL(kern, grid, dim3(64 * kWaves), lds, s, a);
  return hipGetLastError();
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

hipError_t launch_sweep_mfma(const SweepArgs& a, int count, int nt, bool has_h, hipStream_t s) {
  if (a.npad != nt * 32) return hipErrorInvalidValue;
  return has_h ? launch_h<true>(a, count, nt, s) : launch_h<false>(a, count, nt, s);
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
