// Neighbour-triggered flip rate of recorded trajectories (Suppl. "Quantifying
// coupled oscillatory dynamics via neighbor-triggered flip rates"): for every
// step t, over all spins i and trials a of one instance,
//   num(t) = #{(i, a): i flips and some j with J_ij != 0 flips between s(t) and s(t+1)}
//   den(t) = #{(i, a): some j with J_ij != 0 flips},
// so P_NT(t) = num(t) / den(t).  One block per step; adjacency rows and flip
// sets as 256-bit masks.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "internal.hpp"

namespace pim {
namespace {

constexpr int kWords = PIM_MAX_N_LDS / 32;
constexpr int kThreads = 256;

__global__ __launch_bounds__(kThreads) void flip_rate_kernel(FlipRateArgs a) {
  __shared__ uint32_t adj[PIM_MAX_N_LDS][kWords];
  __shared__ unsigned long long red[2][kThreads];
  const int n = a.n;
  for (int e = threadIdx.x; e < PIM_MAX_N_LDS * kWords; e += kThreads) {
    const int i = e / kWords, k = e % kWords;
    uint32_t m = 0;
    if (i < n)
      for (int b = 0; b < 32; ++b) {
        const int j = 32 * k + b;
        if (j < n && j != i && a.j8[(size_t)i * n + j] != 0) m |= 1u << b;
      }
    adj[i][k] = m;
  }
  __syncthreads();
  const int t = blockIdx.x;
  unsigned long long num = 0, den = 0;
  for (int tr = threadIdx.x; tr < a.R; tr += kThreads) {
    const int8_t* s0 = a.trace + ((size_t)tr * (a.T + 1) + t) * a.npad;
    const int8_t* s1 = s0 + a.npad;
    uint32_t f[kWords];
    for (int k = 0; k < kWords; ++k) {
      uint32_t m = 0;
      for (int b = 0; b < 32; ++b) {
        const int j = 32 * k + b;
        if (j < n && s0[j] != s1[j]) m |= 1u << b;
      }
      f[k] = m;
    }
    for (int i = 0; i < n; ++i) {
      uint32_t any = 0;
      for (int k = 0; k < kWords; ++k) any |= adj[i][k] & f[k];
      if (any) {
        ++den;
        num += (f[i >> 5] >> (i & 31)) & 1u;
      }
    }
  }
  red[0][threadIdx.x] = num;
  red[1][threadIdx.x] = den;
  __syncthreads();
  for (int w = kThreads / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w) {
      red[0][threadIdx.x] += red[0][threadIdx.x + w];
      red[1][threadIdx.x] += red[1][threadIdx.x + w];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    a.num[t] = red[0][0];
    a.den[t] = red[1][0];
  }
}

}  // namespace

hipError_t launch_flip_rate(const FlipRateArgs& a, hipStream_t s) {
  if (a.n < 1 || a.n > PIM_MAX_N_LDS || a.T < 1) return hipErrorInvalidValue;
  hipLaunchKernelGGL(flip_rate_kernel, dim3(a.T), dim3(kThreads), 0, s, a);
  return hipGetLastError();
}

}  // namespace pim
