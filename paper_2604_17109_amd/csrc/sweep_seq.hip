// Conventional PIM with sequential updates on the GPU (Box 1, top; Eq. (3)):
// at step t only spin i = t mod N changes, from the local field of the current
// configuration.  Same integer decision table as the parallel kernels (so the
// conventional rule is the table compiled with xi = 0 and uniform noise) and
// the same noise: u is byte i % 16 of the Philox block (i / 16, t, trial,
// stream).
//
// One lane per trial (64 trials per wave, one wave per workgroup), the
// instance's int8 couplings staged in LDS row-major, the trial's spins as int8
// in registers (Npad / 4 words).  A step reads row i of J (broadcast: every
// lane reads the same address), forms I_i = sum_j J_ij s_j + h_i with one
// v_dot4 per four spins, decides, and updates the energy incrementally:
// flipping s_i changes E by 2 s_i(t) I_i(t) (exact integers).
#include <hip/hip_runtime.h>

#include <climits>
#include <cstdint>

#include "internal.hpp"
#include "philox.hpp"

namespace pim {
namespace {

// One wave per workgroup: a trial's steps form one serial dependency chain, so
// the kernel is latency-bound per wave; single-wave workgroups spread the
// trials over as many compute units as there are 64-trial blocks.
constexpr int kWaves = 1;
constexpr int kTabBytes = kTabEntries * 2;

// I_i = sum_j J_ij s_j over one padded row: four independent accumulators so
// the v_dot4 chain is not one serial dependency.
template <int NW>
__device__ __forceinline__ int32_t row_dot(const uint4* row, const uint32_t (&sp)[NW], int32_t init) {
  int32_t acc[4] = {init, 0, 0, 0};
#pragma unroll
  for (int q = 0; q < NW / 4; ++q) {
    const uint4 jv = row[q];
    acc[0] = __builtin_amdgcn_sdot4((int)jv.x, (int)sp[4 * q], acc[0], false);
    acc[1] = __builtin_amdgcn_sdot4((int)jv.y, (int)sp[4 * q + 1], acc[1], false);
    acc[2] = __builtin_amdgcn_sdot4((int)jv.z, (int)sp[4 * q + 2], acc[2], false);
    acc[3] = __builtin_amdgcn_sdot4((int)jv.w, (int)sp[4 * q + 3], acc[3], false);
  }
  return (acc[0] + acc[1]) + (acc[2] + acc[3]);
}

__device__ __forceinline__ int spins_from_bits(uint32_t w) {
  return (int)(0xFFFFFFFFu - 0xFEu * ((w >> 7) & 0x01010101u));
}

template <int NT, bool HAS_H>
__global__ __launch_bounds__(64 * kWaves) void sweep_seq_kernel(SeqArgs a) {
  extern __shared__ __align__(16) unsigned char lds[];
  constexpr int kNpad = NT * 32;
  constexpr int NW = kNpad / 4;  // spin words per trial
  const int inst = blockIdx.y;
  const int wave = threadIdx.x >> 6;
  const int lane = threadIdx.x & 63;
  {
    const uint4* src = reinterpret_cast<const uint4*>(a.j8pad + (size_t)inst * kNpad * kNpad);
    uint4* dst = reinterpret_cast<uint4*>(lds);
    for (int i = threadIdx.x; i < kNpad * kNpad / 16; i += 64 * kWaves) dst[i] = src[i];
  }
  const uint4* sJ = reinterpret_cast<const uint4*>(lds);
  int16_t* sTab = reinterpret_cast<int16_t*>(lds + kNpad * kNpad + wave * kTabBytes);
  uint4* sTab4 = reinterpret_cast<uint4*>(sTab);
  __syncthreads();

  const int tbase = (blockIdx.x * kWaves + wave) * 64;
  if (tbase >= a.R) return;
  const int trial = tbase + lane;
  const bool live = trial < a.R;
  const size_t cell = (size_t)inst * a.R + trial;
  const uint32_t stream = a.inst_stream[inst];
  const int cls = a.inst_class[inst];
  const uint4* gTab4 = reinterpret_cast<const uint4*>(a.thtab + (size_t)cls * a.T * kTabEntries);
  const int32_t* hrow = HAS_H ? a.h + (size_t)inst * kNpad : nullptr;
  const int32_t target = a.target ? a.target[inst] : INT_MIN;
  const int n = a.n;

  // ---- s(0): the same per-spin values as the parallel kernels ----
  uint32_t sp[NW];
#pragma unroll
  for (int q = 0; q < NW / 4; ++q) {
    uint32_t w4[4];
    if (a.init) {
      const uint4 v = live ? *reinterpret_cast<const uint4*>(a.init + cell * kNpad + 16 * q)
                           : uint4{0x01010101u, 0x01010101u, 0x01010101u, 0x01010101u};
      w4[0] = v.x; w4[1] = v.y; w4[2] = v.z; w4[3] = v.w;
    } else {
      const Ctr4 x = philox4x32_10(Ctr4{(uint32_t)q, 0u, (uint32_t)trial, (kDomainInit << 24) | stream}, a.k0, a.k1);
      w4[0] = spins_from_bits(x.x); w4[1] = spins_from_bits(x.y);
      w4[2] = spins_from_bits(x.z); w4[3] = spins_from_bits(x.w);
    }
#pragma unroll
    for (int b = 0; b < 4; ++b) sp[4 * q + b] = w4[b];
  }
  // padded spins (i >= n) meet zero couplings; give them a fixed value
#pragma unroll
  for (int k = 0; k < NW; ++k)
    for (int b = 0; b < 4; ++b)
      if (4 * k + b >= n) sp[k] = (sp[k] & ~(0xFFu << (8 * b))) | (0x01u << (8 * b));

  // ---- E(0) = -1/2 sum_i s_i (I_i + h_i) ----
  int32_t twice = 0;
  for (int i = 0; i < n; ++i) {
    const int32_t acc = row_dot<NW>(sJ + (size_t)i * (kNpad / 16), sp, HAS_H ? hrow[i] : 0);
    const int si = (int)(int8_t)(sp[i >> 2] >> (8 * (i & 3)));
    twice += si * (acc + (HAS_H ? hrow[i] : 0));
  }
  int32_t E = -(twice / 2);
  int32_t e_best = E, t_best = a.start_step, first_hit = (E <= target) ? a.start_step : -1;
  if (live)
#pragma unroll
    for (int k = 0; k < NW; ++k) *reinterpret_cast<uint32_t*>(a.best_s + cell * kNpad + 4 * k) = sp[k];

  int done = a.T;
  sTab4[lane] = gTab4[lane];
  for (int t = 0; t < a.T; ++t) {
    const int tg = a.start_step + t;
    const int i = tg % n;  // wave-uniform
    const uint4 nxt = gTab4[(size_t)min(t + 1, a.T - 1) * 64 + lane];
    // the step's noise block first: its Philox chain overlaps the row product
    const Ctr4 x = philox4x32_10(Ctr4{(uint32_t)(i >> 4), (uint32_t)tg, (uint32_t)trial,
                                      (kDomainNoise << 24) | stream}, a.k0, a.k1);
    const int32_t acc = row_dot<NW>(sJ + (size_t)i * (kNpad / 16), sp, HAS_H ? hrow[i] : 0);
    const int word = i >> 2, sh = 8 * (i & 3);
    // wave-uniform register index (relative addressing of the VGPR array)
    const uint32_t w = sp[word];
    const int s_old = (int)(int8_t)(w >> sh);
    const uint32_t xw = ((i & 15) < 8) ? (((i & 15) < 4) ? x.x : x.y) : (((i & 15) < 12) ? x.z : x.w);
    const int u = (int)((xw >> (8 * (i & 3))) & 0xFFu);
    const int th = sTab[kNoiseVals + (u ^ s_old)];
    const int s_new = (acc >= th) ? 1 : -1;
    if (s_new != s_old) {
      E += 2 * s_old * acc;
      sp[word] = (w & ~(0xFFu << sh)) | ((uint32_t)(s_new & 0xFF) << sh);
    }
    if (E < e_best) {
      e_best = E;
      t_best = tg + 1;
      if (live)
#pragma unroll
        for (int k = 0; k < NW; ++k) *reinterpret_cast<uint32_t*>(a.best_s + cell * kNpad + 4 * k) = sp[k];
    }
    if (first_hit < 0 && E <= target) first_hit = tg + 1;
    if ((t & 1023) == 0 && __atomic_load_n(a.cancel, __ATOMIC_RELAXED) != 0) {
      done = t + 1;
      break;
    }
    // every lookup of this step precedes the table write in the wave's LDS order
    sTab4[lane] = nxt;
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  }
  if (!live) return;
#pragma unroll
  for (int k = 0; k < NW; ++k) *reinterpret_cast<uint32_t*>(a.final_s + cell * kNpad + 4 * k) = sp[k];
  a.e_best[cell] = e_best;
  a.t_best[cell] = t_best;
  a.first_hit[cell] = first_hit;
  a.e_final[cell] = E;
  a.steps_done[cell] = done;
}

template <int NT, bool HAS_H>
hipError_t launch_nt(const SeqArgs& a, int count, hipStream_t s) {
  const size_t lds = (size_t)NT * 32 * NT * 32 + (size_t)kWaves * kTabBytes;
  auto kern = sweep_seq_kernel<NT, HAS_H>;
  hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  const dim3 grid((a.R + 64 * kWaves - 1) / (64 * kWaves), count);
  hipLaunchKernelGGL(kern, grid, dim3(64 * kWaves), lds, s, a);
  return hipGetLastError();
}

template <bool HAS_H>
hipError_t launch_h(const SeqArgs& a, int count, int nt, hipStream_t s) {
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

hipError_t launch_sweep_seq(const SeqArgs& a, int count, int nt, bool has_h, hipStream_t s) {
  if (a.npad != nt * 32 || a.n < 1) return hipErrorInvalidValue;
  return has_h ? launch_h<true>(a, count, nt, s) : launch_h<false>(a, count, nt, s);
}

}  // namespace pim
