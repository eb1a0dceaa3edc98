// Binary64 evaluation of Eq. (1) for candidate configurations (integer
// couplings staged as int8 or FP32, real ones as binary64), and the
// per-instance selection of the lowest-energy trial (the paper's host keeps
// the lowest-energy configuration of all returned states):
//   E = -1/2 (sum_ij s_i J_ij s_j + 2 sum_i h_i s_i).
#include <hip/hip_runtime.h>

#include <cfloat>
#include <climits>
#include <cstdint>

#include "internal.hpp"

namespace pim {
namespace {

constexpr int kWavesPerBlock = 4;

__device__ __forceinline__ double wave_sum(double v) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
  return v;
}

__device__ double config_energy(const float* J, int jstride, const int32_t* h, const int8_t* s, int n,
                                int lane) {
  double acc = 0.0;
  for (int i = 0; i < n; ++i) {
    const double si = (double)s[i];
    const float* Ji = J + (size_t)i * jstride;
    for (int j = lane; j < n; j += 64) acc += si * (double)Ji[j] * (double)s[j];
  }
  if (h)
    for (int j = lane; j < n; j += 64) acc += 2.0 * (double)h[j] * (double)s[j];
  return -0.5 * wave_sum(acc);
}

// Real-valued couplings: binary64 J (row-major n x n) and h.
__device__ double config_energy_real(const double* J, const double* h, const int8_t* s, int n, int lane) {
  double acc = 0.0;
  for (int i = 0; i < n; ++i) {
    const double* Ji = J + (size_t)i * n;
    double row = 0.0;
    for (int j = lane; j < n; j += 64) row += Ji[j] * (double)s[j];
    acc += (double)s[i] * row;
  }
  if (h)
    for (int j = lane; j < n; j += 64) acc += 2.0 * h[j] * (double)s[j];
  return -0.5 * wave_sum(acc);
}

__global__ __launch_bounds__(64 * kWavesPerBlock) void energy_f64_kernel(EnergyArgs a) {
  const int lane = threadIdx.x & 63;
  const int cfg = blockIdx.x * kWavesPerBlock + (threadIdx.x >> 6);
  if (cfg >= a.count) return;
  const int8_t* s = a.spins + (size_t)cfg * a.stride;
  const double e = a.jf64 ? config_energy_real(a.jf64, a.hf64, s, a.n, lane)
                          : config_energy(a.jf32, a.jstride, a.h, s, a.n, lane);
  if (lane == 0) a.out[cfg] = e;
}

// Re-rank for real-valued instances (N <= PIM_MAX_N_LDS): one block per
// (instance, 4 CAND candidates), CAND candidates per wave.  The binary64 J
// streams through LDS in tiles of kRealRows rows, so each row read from L2
// serves all of the block's candidates.  CAND = 8 when that still gives every
// CU a block (large chunks: least L2 traffic), else CAND = 1 (a few requests:
// their candidates spread over more CUs).  Per candidate the arithmetic is config_energy_real's, in the
// same order: lane l sums the columns l, l + 64, ... of each row times the
// spins, then adds s_i times that row sum (binary64, separate multiply and
// add), and the lanes are reduced by wave_sum.  The row's own spin s_i comes
// from the lane holding column i.
constexpr int kRealRows = 16;  // J rows per LDS tile

template <int kRealCand>
__global__ __launch_bounds__(64 * kWavesPerBlock) void rerank_real_kernel(RerankArgs a) {
  __shared__ double sJ[kRealRows][PIM_MAX_N_LDS];
  const int inst = blockIdx.y;
  const int n = a.n, npad = a.npad;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int cand0 = (blockIdx.x * kWavesPerBlock + wave) * kRealCand;
  // spins of columns lane + 64 m (m < 4) of each candidate: packed bytes
  // (for the s_i broadcast) and as binary64 values
  uint32_t packed[kRealCand];
  double sd[kRealCand][4];
#pragma unroll
  for (int c = 0; c < kRealCand; ++c) {
    const int trial = cand0 + c;
    const int8_t* s = a.best_s + ((size_t)inst * a.R + (trial < a.R ? trial : 0)) * npad;
    packed[c] = 0;
#pragma unroll
    for (int m = 0; m < 4; ++m) {
      const int j = lane + 64 * m;
      const int8_t v = (trial < a.R && j < n) ? s[j] : (int8_t)0;
      packed[c] |= (uint32_t)(uint8_t)v << (8 * m);
      sd[c][m] = (double)v;
    }
  }
  const double* J = a.j64[inst];
  double acc[kRealCand];
#pragma unroll
  for (int c = 0; c < kRealCand; ++c) acc[c] = 0.0;
  // thread t stages column t of each tile row (J is row-major n x n, n <= 256
  // = the block size); the next tile's loads are issued before the current
  // tile's arithmetic
  static_assert(64 * kWavesPerBlock == PIM_MAX_N_LDS, "one tile column per thread");
  // (two tiles ahead: the loads of tiles t+1 and t+2 are in flight while
  // tile t is used)
  double nxt[2][kRealRows];
  auto load_tile = [&](int t0, double (&dst)[kRealRows]) {
#pragma unroll
    for (int r = 0; r < kRealRows; ++r)
      dst[r] = (t0 + r < n && (int)threadIdx.x < n) ? J[(size_t)(t0 + r) * n + threadIdx.x] : 0.0;
  };
  load_tile(0, nxt[0]);
  load_tile(kRealRows, nxt[1]);
  for (int t0 = 0; t0 < n; t0 += kRealRows) {
    const int rows = min(kRealRows, n - t0);
    __syncthreads();  // the previous tile has been read
#pragma unroll
    for (int r = 0; r < kRealRows; ++r) sJ[r][threadIdx.x] = nxt[0][r];
    __syncthreads();
#pragma unroll
    for (int r = 0; r < kRealRows; ++r) nxt[0][r] = nxt[1][r];
    if (t0 + 2 * kRealRows < n) load_tile(t0 + 2 * kRealRows, nxt[1]);
#pragma unroll
    for (int r = 0; r < kRealRows; ++r) {
      if (r < rows) {  // uniform
        const int i = t0 + r;
        const int owner = i & 63, shift = 8 * (i >> 6);
#pragma unroll
        for (int c = 0; c < kRealCand; ++c) {
          double row = 0.0;
#pragma unroll
          for (int m = 0; m < 4; ++m) {
            const int j = lane + 64 * m;
            if (j < n) row += sJ[r][j] * sd[c][m];
          }
          const int si = (int)(int8_t)((uint32_t)__builtin_amdgcn_readlane((int)packed[c], owner) >> shift);
          acc[c] += (double)si * row;
        }
      }
    }
  }
  const double* h = a.h64 ? a.h64[inst] : nullptr;
#pragma unroll
  for (int c = 0; c < kRealCand; ++c) {
    double v = acc[c];
    if (h)
#pragma unroll
      for (int m = 0; m < 4; ++m) {
        const int j = lane + 64 * m;
        if (j < n) v += 2.0 * h[j] * sd[c][m];
      }
    const double e = -0.5 * wave_sum(v);
    const int trial = cand0 + c;
    if (lane == 0 && trial < a.R) a.energy[(size_t)inst * a.R + trial] = e;
  }
}

// Batch re-rank of every trial's best state.  One block per (instance, 16
// trials): the instance's int8 couplings are staged in LDS once and each wave
// evaluates four candidates.  Lane l owns columns 4l..4l+3; for every row i
// the exact integer s_i * sum_j J_ij s_j (one v_dot4 per lane) is accumulated
// in binary64, then the lanes are reduced in binary64.
constexpr int kRerankTrialsPerBlock = 16;

__global__ __launch_bounds__(64 * kWavesPerBlock) void rerank_kernel(RerankArgs a) {
  __shared__ __align__(16) int8_t sJ[PIM_MAX_N_LDS * PIM_MAX_N_LDS];
  __shared__ __align__(16) int8_t sS[kWavesPerBlock][PIM_MAX_N_LDS];
  const int inst = blockIdx.y;
  const int n = a.n, npad = a.npad;
  const int8_t* J = a.j8[inst];
  // row stride PIM_MAX_N_LDS; columns >= n are never initialised, which is
  // harmless: the candidate's spins there are 0, so they add 0 to every dot
  for (int i = threadIdx.x; i < n * n; i += 64 * kWavesPerBlock) {
    const int r = i / n, c = i - r * n;
    sJ[r * PIM_MAX_N_LDS + c] = J[i];
  }
  __syncthreads();
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int32_t* hp = a.h ? a.h[inst] : nullptr;
  for (int k = 0; k < kRerankTrialsPerBlock / kWavesPerBlock; ++k) {
    const int trial = blockIdx.x * kRerankTrialsPerBlock + k * kWavesPerBlock + wave;
    if (trial >= a.R) break;  // wave-uniform
    const size_t cell = (size_t)inst * a.R + trial;
    const int8_t* s = a.best_s + cell * npad;
    for (int i = lane; i < PIM_MAX_N_LDS; i += 64) sS[wave][i] = (i < n) ? s[i] : (int8_t)0;
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
    const int32_t s4 = reinterpret_cast<const int32_t*>(sS[wave])[lane];  // columns 4l..4l+3
    double acc = 0.0;
    for (int i = 0; i < n; ++i) {
      const int32_t j4 = reinterpret_cast<const int32_t*>(sJ + i * PIM_MAX_N_LDS)[lane];
      const int dot = __builtin_amdgcn_sdot4(j4, s4, 0, false);  // sum_j J_ij s_j over 4 columns
      acc += (double)(sS[wave][i] * dot);
    }
    if (hp)
      for (int b = 0; b < 4; ++b) {
        const int j = 4 * lane + b;
        if (j < n) acc += 2.0 * (double)hp[j] * (double)sS[wave][j];
      }
    const double e = -0.5 * wave_sum(acc);
    if (lane == 0) a.energy[cell] = e;
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
  }
}

// Re-rank for N > PIM_MAX_N_LDS (couplings too large for LDS): one block per
// (instance, 64 candidates), 16 candidates per wave.  J streams through LDS in
// tiles of kBigRows rows (row stride PIM_MAX_N, columns >= n cleared), so every
// row read from L2 serves all 64 candidates.  Lane l keeps columns 16l ..
// 16l + 15 of its wave's candidates in registers (int8; columns >= n are 0 in
// the LDS rows, so their spins add nothing); a row costs one 16-byte LDS read
// and four v_dot4 per candidate, and the row's own spin s_i comes from the lane
// that holds column i.  Every sum is an exact integer (|s^T J s| <= N^2 * 127
// < 2^31), so the energies equal the binary64 evaluation of Eq. (1) exactly.
constexpr int kBigCand = 16;  // candidates per wave
constexpr int kBigRows = 16;  // J rows per LDS tile

__global__ __launch_bounds__(64 * kWavesPerBlock) void rerank_big_kernel(RerankArgs a) {
  __shared__ __align__(16) int8_t sJ[kBigRows][PIM_MAX_N];
  const int inst = blockIdx.y;
  const int n = a.n, npad = a.npad;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int cand0 = (blockIdx.x * kWavesPerBlock + wave) * kBigCand;
  // this lane's 16 columns of each candidate's state (zero past npad or R)
  const bool has_cols = 16 * lane < npad;
  int4 sv[kBigCand];
#pragma unroll
  for (int c = 0; c < kBigCand; ++c) {
    sv[c] = int4{0, 0, 0, 0};
    const int trial = cand0 + c;
    if (has_cols && trial < a.R)
      sv[c] = *reinterpret_cast<const int4*>(a.best_s + ((size_t)inst * a.R + trial) * npad + 16 * lane);
  }
  for (int i = threadIdx.x; i < kBigRows * PIM_MAX_N / 16; i += 64 * kWavesPerBlock)
    reinterpret_cast<int4*>(&sJ[0][0])[i] = int4{0, 0, 0, 0};
  const int8_t* J = a.j8[inst];
  int acc[kBigCand];
#pragma unroll
  for (int c = 0; c < kBigCand; ++c) acc[c] = 0;
  for (int t0 = 0; t0 < n; t0 += kBigRows) {
    const int rows = min(kBigRows, n - t0);
    __syncthreads();  // the previous tile has been read (and the clearing done)
    // rows t0 .. t0 + rows - 1 are rows * n contiguous bytes of J
    const int8_t* src = J + (size_t)t0 * n;
    for (int k = threadIdx.x; k < rows * n; k += 64 * kWavesPerBlock) {
      const int r = k / n;
      sJ[r][k - r * n] = src[k];
    }
    __syncthreads();
    const int owner = t0 >> 4;  // the lane holding columns t0 .. t0 + 15
#pragma unroll
    for (int r = 0; r < kBigRows; ++r) {
      if (r < rows) {  // uniform
        const int4 jr = has_cols ? *reinterpret_cast<const int4*>(&sJ[r][16 * lane]) : int4{0, 0, 0, 0};
#pragma unroll
        for (int c = 0; c < kBigCand; ++c) {
          int part = __builtin_amdgcn_sdot4(jr.x, sv[c].x, 0, false);
          part = __builtin_amdgcn_sdot4(jr.y, sv[c].y, part, false);
          part = __builtin_amdgcn_sdot4(jr.z, sv[c].z, part, false);
          part = __builtin_amdgcn_sdot4(jr.w, sv[c].w, part, false);
          // s_i of candidate c, i = t0 + r: byte r of the owner lane's columns
          const int w = (r < 4) ? sv[c].x : (r < 8) ? sv[c].y : (r < 12) ? sv[c].z : sv[c].w;
          const int si = (int)(int8_t)(__builtin_amdgcn_readlane(w, owner) >> (8 * (r & 3)));
          acc[c] += si * part;
        }
      }
    }
  }
  const int32_t* hp = a.h ? a.h[inst] : nullptr;
#pragma unroll
  for (int c = 0; c < kBigCand; ++c) {
    const int trial = cand0 + c;
    // the field term 2 sum_j h_j s_j over this lane's columns, in binary64
    double hs = 0.0;
    if (hp && has_cols) {
      const int q[4] = {sv[c].x, sv[c].y, sv[c].z, sv[c].w};
#pragma unroll
      for (int b = 0; b < 16; ++b) {
        const int j = 16 * lane + b;
        if (j < n) hs += 2.0 * (double)hp[j] * (double)(int8_t)(q[b >> 2] >> (8 * (b & 3)));
      }
    }
    const double e = -0.5 * wave_sum((double)acc[c] + hs);
    if (lane == 0 && trial < a.R) a.energy[(size_t)inst * a.R + trial] = e;
  }
}

// One block per instance: lowest binary64 energy, ties to the lowest trial;
// gathers that trial's state, step and tracked integer energy.
__global__ __launch_bounds__(256) void select_best_kernel(RerankArgs a) {
  __shared__ double se[256];
  __shared__ int st[256];
  const int inst = blockIdx.x;
  double best = DBL_MAX;
  int arg = INT_MAX;
  for (int r = threadIdx.x; r < a.R; r += 256) {
    const double e = a.energy[(size_t)inst * a.R + r];
    if (e < best || (e == best && r < arg)) {
      best = e;
      arg = r;
    }
  }
  se[threadIdx.x] = best;
  st[threadIdx.x] = arg;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) {
      const double e2 = se[threadIdx.x + w];
      const int a2 = st[threadIdx.x + w];
      if (e2 < se[threadIdx.x] || (e2 == se[threadIdx.x] && a2 < st[threadIdx.x])) {
        se[threadIdx.x] = e2;
        st[threadIdx.x] = a2;
      }
    }
    __syncthreads();
  }
  const int bt = st[0];
  const size_t cell = (size_t)inst * a.R + bt;
  for (int i = threadIdx.x; i < a.npad; i += 256) a.out_spins[(size_t)inst * a.npad + i] = a.best_s[cell * a.npad + i];
  if (threadIdx.x == 0) {
    a.out_energy[inst] = se[0];
    a.out_trial[inst] = bt;
    a.out_step[inst] = a.t_best[cell];
    a.out_tracked[inst] = a.e_best[cell];
  }
}

}  // namespace

hipError_t launch_energy_f64(const EnergyArgs& a, hipStream_t s) {
  if (a.count < 1) return hipSuccess;
  const dim3 grid((a.count + kWavesPerBlock - 1) / kWavesPerBlock);
  hipLaunchKernelGGL(energy_f64_kernel, grid, dim3(64 * kWavesPerBlock), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_rerank_select(const RerankArgs& a, hipStream_t s) {
  if (a.n > PIM_MAX_N) return hipErrorInvalidValue;
  if (a.j64) {
    if (a.n > PIM_MAX_N_LDS) return hipErrorInvalidValue;
    constexpr int kWide = 8, kCus = 256;
    const size_t wide_blocks = (size_t)a.count * ((a.R + kWavesPerBlock * kWide - 1) / (kWavesPerBlock * kWide));
    if (wide_blocks >= kCus) {
      const dim3 grid((a.R + kWavesPerBlock * kWide - 1) / (kWavesPerBlock * kWide), a.count);
      hipLaunchKernelGGL(rerank_real_kernel<kWide>, grid, dim3(64 * kWavesPerBlock), 0, s, a);
    } else {
      const dim3 grid((a.R + kWavesPerBlock - 1) / kWavesPerBlock, a.count);
      hipLaunchKernelGGL(rerank_real_kernel<1>, grid, dim3(64 * kWavesPerBlock), 0, s, a);
    }
  } else if (a.n > PIM_MAX_N_LDS) {
    if (a.npad > PIM_MAX_N || a.npad % 16) return hipErrorInvalidValue;
    const int per_block = kWavesPerBlock * kBigCand;
    const dim3 grid((a.R + per_block - 1) / per_block, a.count);
    hipLaunchKernelGGL(rerank_big_kernel, grid, dim3(64 * kWavesPerBlock), 0, s, a);
  } else {
    const dim3 grid((a.R + kRerankTrialsPerBlock - 1) / kRerankTrialsPerBlock, a.count);
    hipLaunchKernelGGL(rerank_kernel, grid, dim3(64 * kWavesPerBlock), 0, s, a);
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(select_best_kernel, dim3(a.count), dim3(256), 0, s, a);
  return hipGetLastError();
}

}  // namespace pim
