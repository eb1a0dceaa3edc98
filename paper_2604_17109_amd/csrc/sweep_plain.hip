// Plain FP32 PIMI sweep: one instance per launch, no matrix cores.
//
// Workgroup = 32 trials x (ceil(N/16) spin blocks); thread (b, a) owns spins
// 16b..16b+15 of trial a.  Each step it forms the 16 local fields (Eq. (2))
// with ordinary FP32 multiply-adds over float4 chunks of J rows (zero-padded to
// whole rows of 16 and a multiple of 4 columns) and of the trial's current
// spins (LDS), one spin chunk reused across the 16 rows.  J is staged in LDS
// once when its padded rows fit (up to 120 KB, N <= 172), and read from
// global memory (L2) otherwise.  It then applies the
// same integer-threshold form of Eq. (4) as the MFMA kernel:
// k = #{j : I >= theta_j}, s' = +1 iff u >= umin[2k + (s<0)].  FP32 sums of
// integers below 2^24 are exact, so both kernels produce identical
// trajectories.
//
// Real-valued instances use the same kernel with binary32 fields I = sum_j
// fl32(J_ij) s_j + fl32(h_i), binary32 thresholds (smallest binary32 field that
// reaches each LUT breakpoint under the binary64 rule) and binary32 energies
// reduced in a fixed order.
#include <hip/hip_runtime.h>

#include <climits>
#include <cmath>
#include <cstdint>

#include "internal.hpp"
#include "philox.hpp"

namespace pim {
namespace {

constexpr int kTrials = 32;
constexpr int kBlocks = PIM_MAX_N_LDS / 16;  // spin blocks of 16
constexpr int kThreads = kTrials * kBlocks;
constexpr int kRow = PIM_MAX_N_LDS + 8;      // LDS row stride (floats) of one trial's spins
constexpr size_t kJLdsMax = 120 * 1024;      // largest J staged in LDS (bytes)

// bytes of J's padded rows 0 .. 16 ceil(n/16) - 1
size_t plain_j_bytes(const PlainArgs& a) { return (size_t)16 * ((a.n + 15) / 16) * a.jstride * 4; }

template <bool REAL, bool JLDS>
__global__ __launch_bounds__(kThreads) void sweep_plain_kernel(PlainArgs a) {
  __shared__ __align__(16) float sS[kTrials][kRow];
  __shared__ int32_t sE[kTrials];
  __shared__ float sEf[kBlocks][kTrials];  // per-block partial energies (REAL)
  extern __shared__ __align__(16) float sJ[];  // J rows (JLDS)
  // blockDim = 32 x nb: every thread owns a spin block
  const int b = threadIdx.x / kTrials;
  const int al = threadIdx.x % kTrials;
  const int trial = blockIdx.x * kTrials + al;
  const bool live = trial < a.R;
  const int nb = (a.n + 15) / 16;
  const bool owner = b < nb;
  if (JLDS) {
    const float4* src = reinterpret_cast<const float4*>(a.jf32);
    float4* dst = reinterpret_cast<float4*>(sJ);
    const int n4 = 16 * nb * a.jstride / 4;
    for (int i = threadIdx.x; i < n4; i += blockDim.x) dst[i] = src[i];
  }
  const size_t cell = (size_t)trial;
  const int L = a.levels;
  const int w = (L - 1) + 2 * L;

  // s(0)
  if (owner) {
    if (a.init) {
      for (int q = 0; q < 16; ++q) {
        const int i = 16 * b + q;
        // clamped address: no load outside the trial's row even if speculated
        const float v = (float)a.init[(live ? cell : 0) * a.npad + min(i, a.n - 1)];
        sS[al][i] = (live && i < a.n) ? v : 1.0f;
      }
    } else {
      const Ctr4 x = philox4x32_10(Ctr4{(uint32_t)b, 0u, (uint32_t)trial, (kDomainInit << 24) | a.stream}, a.k0, a.k1);
      const uint32_t xw[4] = {x.x, x.y, x.z, x.w};
      for (int q = 0; q < 16; ++q) {
        const uint32_t u = (xw[q >> 2] >> (8 * (q & 3))) & 0xFFu;
        sS[al][16 * b + q] = u >= 128u ? 1.0f : -1.0f;
      }
    }
  }
  if (threadIdx.x < kTrials) sE[threadIdx.x] = 0;
  __syncthreads();

  int32_t e_best = INT_MAX, t_best = -1, first_hit = -1, e_cur = 0;
  float ef_best = INFINITY, ef_cur = 0.0f;
  float target_f;
  __builtin_memcpy(&target_f, &a.target, 4);
  int done = a.T;
  for (int t = 0;; ++t) {
    const int tg = a.start_step + t;
    float I[16];
    float s_old[16];
    if (owner) {
#pragma unroll
      for (int q = 0; q < 16; ++q) I[q] = 0.0f;
      const int n4 = a.jstride;
      const float4* S4 = reinterpret_cast<const float4*>(&sS[al][0]);
      // rows are zero-padded to a multiple of 32 and columns to jstride, so
      // every row of the block exists and padded columns add 0
      const float* Jb = (JLDS ? sJ : a.jf32) + (size_t)(16 * b) * n4;
      for (int j4 = 0; j4 < n4 / 4; ++j4) {
        const float4 sv = S4[j4];
#pragma unroll
        for (int q = 0; q < 16; ++q) {
          const float4 jv = *reinterpret_cast<const float4*>(Jb + (size_t)q * n4 + 4 * j4);
          I[q] = fmaf(jv.x, sv.x, I[q]);
          I[q] = fmaf(jv.y, sv.y, I[q]);
          I[q] = fmaf(jv.z, sv.z, I[q]);
          I[q] = fmaf(jv.w, sv.w, I[q]);
        }
      }
      int32_t ep = 0;
      float epf = 0.0f;
#pragma unroll
      for (int q = 0; q < 16; ++q) {
        const int i = 16 * b + q;
        s_old[q] = sS[al][i];
        if (REAL) {
          const float hv = (a.hf && i < a.n) ? a.hf[min(i, a.n - 1)] : 0.0f;
          I[q] += hv;
          if (i < a.n) epf += s_old[q] * (I[q] + hv);
        } else {
          const int hv = (a.h && i < a.n) ? a.h[min(i, a.n - 1)] : 0;
          I[q] += (float)hv;
          if (i < a.n) ep += (int32_t)s_old[q] * ((int32_t)I[q] + hv);
        }
      }
      if (REAL) sEf[b][al] = epf;
      else atomicAdd(&sE[al], ep);
    } else if (REAL) {
      sEf[b][al] = 0.0f;
    }
    __syncthreads();
    bool improved;
    if (REAL) {
      float tot = 0.0f;
      for (int k = 0; k < nb; ++k) tot += sEf[k][al];  // fixed order
      // the blocks past nb contributed +0.0 (turns a -0.0 sum into +0.0)
      if (nb < kBlocks) tot += 0.0f;
      const float E = -0.5f * tot;
      improved = E < ef_best;
      if (improved) ef_best = E;
      if (a.use_target && first_hit < 0 && E <= target_f) first_hit = tg;
      ef_cur = E;
    } else {
      const int32_t E = -(sE[al] / 2);
      improved = E < e_best;
      if (improved) e_best = E;
      if (a.use_target && first_hit < 0 && E <= a.target) first_hit = tg;
      e_cur = E;
    }
    if (improved) {
      t_best = tg;
      if (owner && live)
        for (int q = 0; q < 16; ++q) {
          const int i = 16 * b + q;
          if (i < a.npad) a.best_s[cell * a.npad + i] = (int8_t)s_old[q];
        }
    }
    if (t == a.T) break;
    if ((t & 255) == 0 && __atomic_load_n(a.cancel, __ATOMIC_RELAXED) != 0) {
      done = t;
      break;
    }
    float s_new[16];
    if (owner) {
      const int32_t* row = a.steptab + (size_t)t * w;
      const Ctr4 x = philox4x32_10(Ctr4{(uint32_t)b, (uint32_t)tg, (uint32_t)trial, (kDomainNoise << 24) | a.stream},
                                   a.k0, a.k1);
      const uint32_t xw[4] = {x.x, x.y, x.z, x.w};
#pragma unroll
      for (int q = 0; q < 16; ++q) {
        int k = 0;
        for (int j = 0; j < L - 1; ++j) k += (I[q] >= (REAL ? __int_as_float(row[j]) : (float)row[j])) ? 1 : 0;
        const int sneg = s_old[q] < 0.0f ? 1 : 0;
        const int umin = row[(L - 1) + 2 * k + sneg];
        const int u = (int)((xw[q >> 2] >> (8 * (q & 3))) & 0xFFu);
        s_new[q] = (u >= umin) ? 1.0f : -1.0f;
      }
    }
    __syncthreads();  // every thread has read the old spins and E
    if (owner)
#pragma unroll
      for (int q = 0; q < 16; ++q) sS[al][16 * b + q] = s_new[q];
    if (threadIdx.x < kTrials) sE[threadIdx.x] = 0;
    __syncthreads();
  }

  if (owner && live)
    for (int q = 0; q < 16; ++q) {
      const int i = 16 * b + q;
      if (i < a.npad) a.final_s[cell * a.npad + i] = (int8_t)sS[al][i];
    }
  if (b == 0 && live) {
    a.e_best[cell] = REAL ? __float_as_int(ef_best) : e_best;
    a.t_best[cell] = t_best;
    a.first_hit[cell] = first_hit;
    a.e_final[cell] = REAL ? __float_as_int(ef_cur) : e_cur;
    a.steps_done[cell] = done;
  }
}

}  // namespace

template <bool REAL, bool JLDS>
hipError_t launch_plain(const PlainArgs& a, hipStream_t s) {
  const size_t lds = JLDS ? plain_j_bytes(a) : 0;
  auto kern = sweep_plain_kernel<REAL, JLDS>;
  if (JLDS) {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)kJLdsMax);
    if (e != hipSuccess) return e;
  }
  const dim3 grid((a.R + kTrials - 1) / kTrials);
  hipLaunchKernelGGL(kern, grid, dim3(kTrials * ((a.n + 15) / 16)), lds, s, a);
  return hipGetLastError();
}

hipError_t launch_sweep_plain(const PlainArgs& a, bool real, hipStream_t s) {
  if (a.n > PIM_MAX_N_LDS || a.n < 1) return hipErrorInvalidValue;
  const bool jlds = plain_j_bytes(a) <= kJLdsMax;
  if (real) return jlds ? launch_plain<true, true>(a, s) : launch_plain<true, false>(a, s);
  return jlds ? launch_plain<false, true>(a, s) : launch_plain<false, false>(a, s);
}

}  // namespace pim
