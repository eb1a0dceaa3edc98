// Binary64 re-evaluation of Eq. (1) for candidate configurations: one
// workgroup per configuration, E = -1/2 sum_i s_i (sum_j J_ij s_j + 2 h_i).
#include <hip/hip_runtime.h>

#include <cstdint>

#include "internal.hpp"

namespace pim {
namespace {

constexpr int kThreads = 256;

__global__ __launch_bounds__(kThreads) void energy_f64_kernel(EnergyArgs a) {
  __shared__ double part[kThreads / 64];
  const int8_t* s = a.spins + (size_t)blockIdx.x * a.stride;
  double acc = 0.0;
  for (int i = threadIdx.x; i < a.n; i += kThreads) {
    double row = 0.0;
    const float* Ji = a.jf32 + (size_t)i * a.n;
    for (int j = 0; j < a.n; ++j) row += (double)Ji[j] * (double)s[j];
    const double hv = a.h ? (double)a.h[i] : 0.0;
    acc += (double)s[i] * (row + 2.0 * hv);
  }
  for (int off = 32; off > 0; off >>= 1) acc += __shfl_down(acc, off);
  if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    double tot = 0.0;
    for (int k = 0; k < kThreads / 64; ++k) tot += part[k];
    a.out[blockIdx.x] = -0.5 * tot;
  }
}

}  // namespace

hipError_t launch_energy_f64(const EnergyArgs& a, hipStream_t s) {
  if (a.count < 1) return hipSuccess;
  hipLaunchKernelGGL(energy_f64_kernel, dim3(a.count), dim3(kThreads), 0, s, a);
  return hipGetLastError();
}

}  // namespace pim
