// MIMO detection as an Ising problem, built on the device in binary64.
//
// The same mapping as the host's pim_mimo_ising (Suppl. "MIMO problem
// definition", "Real-Valued equivalent", "Delta-Ising MIMO (DI-MIMO)
// formulation", "Baseline: linear MMSE detector"), one workgroup per request:
//
//   Hr = [[Re H, -Im H], [Im H, Re H]] (2Nr x 2Nt),  yr = [Re y; Im y],
//   G  = Hr^T Hr,
//   x_m = 0 (ML) or slice((G + I / esn0)^-1 Hr^T yr) (DI; Cholesky),
//   r  = yr - Hr x_m,  c = Hr^T r,
//   J  = -2 w_a w_b G_ij off the diagonal (spin a*2Nt + i carries weight w_a
//        on real component i),  h = 2 w_a c_i.
//
// Hr is never formed: its entries are read from the complex H (interleaved
// (re, im), row-major Nr x Nt), which is staged in LDS when it fits beside the
// lower triangle of G.  Every sum runs over its index in ascending order with
// separate multiplies and adds, as the host function does; the Cholesky
// factor is formed right-looking, which applies each element's subtractions in
// that same order, so G, J and the factor equal the host's bit for bit.  The
// triangular solves run in one wave (lane l owns rows l and l + 64).
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstring>
#include <vector>

#include "internal.hpp"

namespace pim {
namespace {

constexpr int kThreads = 1024;  // 4 waves per SIMD: the LDS-latency-bound loops overlap
constexpr size_t kLdsLimit = 160 * 1024;  // LDS per workgroup on gfx950

__device__ __forceinline__ double hr_at(const double* H, int nr, int nt, int k, int j) {
  // element (k, j) of the real-valued equivalent
  const bool lo_row = k < nr, lo_col = j < nt;
  const int kk = lo_row ? k : k - nr, jj = lo_col ? j : j - nt;
  const double re = H[2 * (kk * nt + jj)], im = H[2 * (kk * nt + jj) + 1];
  if (lo_row) return lo_col ? re : -im;
  return lo_col ? im : re;
}

__device__ __forceinline__ double yr_at(const double* y, int nr, int k) {
  return k < nr ? y[2 * k] : y[2 * (k - nr) + 1];
}

__device__ __forceinline__ double slice_level(double v, int qam) {
  const double m = qam == 4 ? 1.0 : 3.0;
  const double q = 2.0 * floor(v / 2.0) + 1.0;
  return q < -m ? -m : (q > m ? m : q);
}

// packed lower triangle: (i, j), j <= i
__device__ __forceinline__ int tri(int i, int j) { return i * (i + 1) / 2 + j; }

// Column i of Hr as (offset of its re/im value in H, sign) for the rows
// k < nr (first) and k >= nr (second); the row stride in H is 2 nt.
struct HrCol {
  int off_lo, off_hi;
  double sg_lo, sg_hi;
};
__device__ __forceinline__ HrCol hr_col(int nt, int i) {
  // Hr[k][i] = Re H[k][i] (k < nr), Im H[k-nr][i] (k >= nr) for i < nt;
  //          = -Im H[k][i-nt] (k < nr), Re H[k-nr][i-nt] (k >= nr) otherwise
  if (i < nt) return HrCol{2 * i, 2 * i + 1, 1.0, 1.0};
  return HrCol{2 * (i - nt) + 1, 2 * (i - nt), -1.0, 1.0};
}

template <bool STAGE_H>
__global__ __launch_bounds__(kThreads) void mimo_map_kernel(MimoMapArgs a) {
  extern __shared__ __align__(16) double smem[];
  __shared__ int bad;
  const int slot = blockIdx.x;
  if (slot >= a.count) return;
  const int tid = threadIdx.x;
  const MimoSlot rec = a.slots[slot];
  const int nr = rec.nr, nt = rec.nt, qam = rec.qam, map = rec.map;
  const int m = 2 * nr, n2 = 2 * nt;
  const int nb = (map == PIM_MIMO_ML && qam == 4) ? 1 : 2;
  const double w0 = (map == PIM_MIMO_ML && qam == 16) ? 2.0 : 1.0, w1 = 1.0;
  const int n = nb * n2;
  const double* Hg = a.hy + rec.hy_off;
  double* J = a.j64 + (size_t)slot * a.npad * a.npad;
  double* hv = a.h64 + (size_t)slot * a.npad;
  double* xm_out = a.xm + (size_t)slot * a.xm_stride;

  // LDS: [H, y (staged)] | G lower triangle | z [n2] | x_m [n2] | r [m] | c [n2]
  const int hy_len = STAGE_H ? 2 * nr * nt + 2 * nr : 0;
  double* G = smem + hy_len;
  double* z = G + n2 * (n2 + 1) / 2;
  double* xm = z + n2;
  double* r = xm + n2;
  double* c = r + m;
  if (STAGE_H)
    for (int i = tid; i < hy_len; i += kThreads) smem[i] = Hg[i];
  if (tid == 0) bad = 0;
  __syncthreads();
  const double* Hs = STAGE_H ? smem : Hg;
  const double* ys = Hs + 2 * nr * nt;

  // ---- G = Hr^T Hr, lower triangle: each thread a 4 x 4 block of entries
  //      (rows 4 bi.., columns 4 bj.., bi >= bj), every entry summed over k in
  //      ascending order as above ----
  {
    const int nb4 = (n2 + 3) / 4;
    for (int t = tid; t < nb4 * nb4; t += kThreads) {
      const int bi = t / nb4, bj = t % nb4;
      if (bj > bi) continue;
      HrCol ci[4], cj[4];
      for (int q = 0; q < 4; ++q) {
        ci[q] = hr_col(nt, min(4 * bi + q, n2 - 1));
        cj[q] = hr_col(nt, min(4 * bj + q, n2 - 1));
      }
      double acc[4][4];
      for (int a = 0; a < 4; ++a)
        for (int b = 0; b < 4; ++b) acc[a][b] = 0.0;
      for (int k = 0; k < nr; ++k) {  // rows k < nr of Hr
        const double* row = Hs + 2 * k * nt;
        double x[4], y[4];
        for (int q = 0; q < 4; ++q) {
          x[q] = ci[q].sg_lo * row[ci[q].off_lo];
          y[q] = cj[q].sg_lo * row[cj[q].off_lo];
        }
        for (int a = 0; a < 4; ++a)
          for (int b = 0; b < 4; ++b) acc[a][b] += x[a] * y[b];
      }
      for (int k = 0; k < nr; ++k) {  // rows k >= nr
        const double* row = Hs + 2 * k * nt;
        double x[4], y[4];
        for (int q = 0; q < 4; ++q) {
          x[q] = ci[q].sg_hi * row[ci[q].off_hi];
          y[q] = cj[q].sg_hi * row[cj[q].off_hi];
        }
        for (int a = 0; a < 4; ++a)
          for (int b = 0; b < 4; ++b) acc[a][b] += x[a] * y[b];
      }
      for (int a = 0; a < 4; ++a)
        for (int b = 0; b < 4; ++b) {
          const int i = 4 * bi + a, j = 4 * bj + b;
          if (i < n2 && j <= i) G[tri(i, j)] = acc[a][b];
        }
    }
  }
  __syncthreads();
  // ---- J from G (zero diagonal, zero padding to npad x npad) ----
  for (int e = tid; e < a.npad * a.npad; e += kThreads) {
    const int p = e / a.npad, q = e % a.npad;
    double v = 0.0;
    if (p < n && q < n && p != q) {
      const int pa = p / n2, i = p % n2, qb = q / n2, j = q % n2;
      v = -2.0 * (pa ? w1 : w0) * (qb ? w1 : w0) * G[i >= j ? tri(i, j) : tri(j, i)];
    }
    J[e] = v;
  }
  // ---- x_m ----
  if (map == PIM_MIMO_DI) {
    for (int i = tid; i < n2; i += kThreads) {  // b = Hr^T yr
      const HrCol a = hr_col(nt, i);
      double v = 0.0;
      for (int k = 0; k < nr; ++k) v += (a.sg_lo * Hs[2 * k * nt + a.off_lo]) * ys[2 * k];
      for (int k = 0; k < nr; ++k) v += (a.sg_hi * Hs[2 * k * nt + a.off_hi]) * ys[2 * k + 1];
      z[i] = v;
    }
    __syncthreads();  // J has read G: it becomes A = G + I / esn0, factored in place
    for (int i = tid; i < n2; i += kThreads) G[tri(i, i)] += 1.0 / rec.esn0;
    __syncthreads();
    // Cholesky A = L L^T, right-looking, two phases per column: (1) every
    // thread forms the pivot sqrt(A_jj) itself and the rows below j are
    // divided by it; (2) the trailing update A_ik -= L_ij L_kj (j < k <= i) on
    // a 32 x 32 thread grid.  A pivot that is not positive (A not positive
    // definite in binary64) marks the request as failed.
    const int tr = tid >> 5, tc = tid & 31;
    for (int j = 0; j < n2; ++j) {
      double d = G[tri(j, j)];
      if (!(d > 0.0)) {
        if (tid == 0) bad = 1;
        d = 1.0;
      }
      const double djj = sqrt(d);
      for (int i = j + 1 + tid; i < n2; i += kThreads) G[tri(i, j)] = G[tri(i, j)] / djj;
      __syncthreads();
      if (tid == 0) G[tri(j, j)] = djj;
      // this thread's rows i = j+1+tr+32a and columns k = j+1+tc+32b (k <= i):
      // operands loaded first, so the reads overlap, then updated
      double lik[4], lkj[4], aik[4][4];
      for (int q = 0; q < 4; ++q) {
        const int i = j + 1 + tr + 32 * q, k = j + 1 + tc + 32 * q;
        lik[q] = i < n2 ? G[tri(i, j)] : 0.0;
        lkj[q] = k < n2 ? G[tri(k, j)] : 0.0;
      }
      for (int qa = 0; qa < 4; ++qa)
        for (int qb = 0; qb <= qa; ++qb) {
          const int i = j + 1 + tr + 32 * qa, k = j + 1 + tc + 32 * qb;
          aik[qa][qb] = (i < n2 && k <= i) ? G[tri(i, k)] : 0.0;
        }
      for (int qa = 0; qa < 4; ++qa)
        for (int qb = 0; qb <= qa; ++qb) {
          const int i = j + 1 + tr + 32 * qa, k = j + 1 + tc + 32 * qb;
          if (i < n2 && k <= i) G[tri(i, k)] = aik[qa][qb] - lik[qa] * lkj[qb];
        }
      __syncthreads();
    }
    // L w = b, then L^T z = w, in wave 0: lane l owns rows l and l + 64
    if (tid < 64) {
      double zr[2];
      for (int q = 0; q < 2; ++q) zr[q] = (tid + 64 * q < n2) ? z[tid + 64 * q] : 0.0;
      for (int k = 0; k < n2; ++k) {  // forward: z_k is final once divided; the rows below subtract it
        const double zk = __shfl(zr[k >> 6], k & 63) / G[tri(k, k)];
        for (int q = 0; q < 2; ++q) {
          const int i = tid + 64 * q;
          if (i == k) zr[q] = zk;
          else if (i > k && i < n2) zr[q] = zr[q] - G[tri(i, k)] * zk;
        }
      }
      for (int k = n2 - 1; k >= 0; --k) {  // backward
        const double zk = __shfl(zr[k >> 6], k & 63) / G[tri(k, k)];
        for (int q = 0; q < 2; ++q) {
          const int i = tid + 64 * q;
          if (i == k) zr[q] = zk;
          else if (i < k) zr[q] = zr[q] - G[tri(k, i)] * zk;
        }
      }
      for (int q = 0; q < 2; ++q)
        if (tid + 64 * q < n2) z[tid + 64 * q] = zr[q];
    }
    __syncthreads();
    // a failed request: x_m and h are NaN, so its binary64 energy is NaN
    for (int i = tid; i < n2; i += kThreads) xm[i] = bad ? NAN : slice_level(z[i], qam);
  } else {
    for (int i = tid; i < n2; i += kThreads) xm[i] = 0.0;
  }
  __syncthreads();
  // ---- r = yr - Hr x_m, c = Hr^T r, h ----
  for (int k = tid; k < m; k += kThreads) {
    double v = yr_at(ys, nr, k);
    for (int j = 0; j < n2; ++j) v -= hr_at(Hs, nr, nt, k, j) * xm[j];
    r[k] = v;
  }
  __syncthreads();
  for (int i = tid; i < n2; i += kThreads) {
    const HrCol a = hr_col(nt, i);
    double v = 0.0;
    for (int k = 0; k < nr; ++k) v += (a.sg_lo * Hs[2 * k * nt + a.off_lo]) * r[k];
    for (int k = 0; k < nr; ++k) v += (a.sg_hi * Hs[2 * k * nt + a.off_hi]) * r[nr + k];
    c[i] = v;
  }
  __syncthreads();
  for (int p = tid; p < a.npad; p += kThreads) hv[p] = p < n ? 2.0 * ((p / n2) ? w1 : w0) * c[p % n2] : 0.0;
  for (int i = tid; i < a.xm_stride; i += kThreads) xm_out[i] = i < n2 ? xm[i] : 0.0;
}

}  // namespace

size_t mimo_map_work_doubles(int nr, int nt) {
  // LDS doubles of one request besides its staged H and y: G triangle, z, x_m, r, c
  const size_t n2 = 2 * (size_t)nt, m = 2 * (size_t)nr;
  return n2 * (n2 + 1) / 2 + 3 * n2 + m;
}

hipError_t launch_mimo_map(const MimoMapArgs& a, size_t max_work, size_t max_hy, hipStream_t s) {
  // max_work / max_hy: the largest mimo_map_work_doubles and H + y doubles
  // among the launch's requests (they size the LDS); H and y are staged in
  // LDS when both fit
  if (a.count < 1) return hipSuccess;
  const size_t staged = (max_work + max_hy) * sizeof(double);
  const bool stage = staged <= kLdsLimit;
  const size_t lds = stage ? staged : max_work * sizeof(double);
  if (lds > kLdsLimit) return hipErrorInvalidValue;
  const void* k = stage ? reinterpret_cast<const void*>(mimo_map_kernel<true>)
                        : reinterpret_cast<const void*>(mimo_map_kernel<false>);
  hipError_t e = hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  if (stage) hipLaunchKernelGGL(mimo_map_kernel<true>, dim3(a.count), dim3(kThreads), lds, s, a);
  else hipLaunchKernelGGL(mimo_map_kernel<false>, dim3(a.count), dim3(kThreads), lds, s, a);
  return hipGetLastError();
}

}  // namespace pim

using namespace pim;

extern "C" pim_status pim_mimo_ising_device(const double* Hc, const double* yc, int32_t nr, int32_t nt, int32_t qam,
                                            int32_t map, double esn0, double* J, double* h, double* xm,
                                            int32_t* n_out, void* stream) {
  try {
    if (!Hc || !yc || !J || !h || !xm || !n_out) return fail(PIM_ERR_INVALID, "NULL argument");
    if (qam != 4 && qam != 16) return fail(PIM_ERR_UNSUPPORTED, "qam = %d (4 and 16 are implemented)", qam);
    if (map != PIM_MIMO_ML && map != PIM_MIMO_DI) return fail(PIM_ERR_INVALID, "unknown mapping %d", map);
    if (nt < 1 || 4 * nt > PIM_MAX_N_LDS || nr < 1 || 2 * nr > PIM_MAX_N_LDS)
      return fail(PIM_ERR_INVALID, "nr = %d, nt = %d: need 1 <= nt <= %d and 1 <= nr <= %d", nr, nt,
                  PIM_MAX_N_LDS / 4, PIM_MAX_N_LDS / 2);
    if (map == PIM_MIMO_DI && !(std::isfinite(esn0) && esn0 > 0.0))
      return fail(PIM_ERR_INVALID, "esn0 must be finite and > 0 for the DI mapping");
    const size_t nh = 2 * (size_t)nr * nt, ny = 2 * (size_t)nr;
    for (size_t i = 0; i < nh; ++i)
      if (!std::isfinite(Hc[i])) return fail(PIM_ERR_INVALID, "H is not finite");
    for (size_t i = 0; i < ny; ++i)
      if (!std::isfinite(yc[i])) return fail(PIM_ERR_INVALID, "y is not finite");
    const int n = (map == PIM_MIMO_ML && qam == 4) ? 2 * nt : 4 * nt;
    const int np = 32 * ((n + 31) / 32);
    const int xs = PIM_MAX_N_LDS / 2;
    hipStream_t s = (hipStream_t)stream;
    // one allocation: slot record | H, y | J | h | x_m
    const size_t o_hy = 256, o_j = o_hy + ((nh + ny) * 8 + 255) / 256 * 256;
    const size_t o_h = o_j + (size_t)np * np * 8, o_x = o_h + (size_t)np * 8, total = o_x + (size_t)xs * 8;
    uint8_t* d = static_cast<uint8_t*>(dev_alloc(total, s));
    if (!d) return fail(PIM_ERR_NOMEM, "device allocation of %zu bytes failed", total);
    std::vector<uint8_t> up(o_j, 0);
    const MimoSlot rec{nr, nt, qam, map, esn0, 0};
    std::memcpy(up.data(), &rec, sizeof rec);
    std::memcpy(up.data() + o_hy, Hc, nh * 8);
    std::memcpy(up.data() + o_hy + nh * 8, yc, ny * 8);
    MimoMapArgs a{};
    a.slots = reinterpret_cast<const MimoSlot*>(d);
    a.hy = reinterpret_cast<const double*>(d + o_hy);
    a.j64 = reinterpret_cast<double*>(d + o_j);
    a.h64 = reinterpret_cast<double*>(d + o_h);
    a.xm = reinterpret_cast<double*>(d + o_x);
    a.npad = np;
    a.xm_stride = xs;
    a.count = 1;
    std::vector<double> Jp((size_t)np * np), hp(np), xp(xs);
    hipError_t e = hipMemcpyAsync(d, up.data(), up.size(), hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = launch_mimo_map(a, mimo_map_work_doubles(nr, nt), nh + ny, s);
    if (e == hipSuccess) e = hipMemcpyAsync(Jp.data(), d + o_j, Jp.size() * 8, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipMemcpyAsync(hp.data(), d + o_h, hp.size() * 8, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipMemcpyAsync(xp.data(), d + o_x, xp.size() * 8, hipMemcpyDeviceToHost, s);
    hipError_t es = hipStreamSynchronize(s);
    if (e == hipSuccess) e = es;
    dev_free(d, s);
    if (e != hipSuccess) return fail(PIM_ERR_DEVICE, "pim_mimo_ising_device failed: %s", hipGetErrorString(e));
    if (map == PIM_MIMO_DI && std::isnan(xp[0]))
      return fail(PIM_ERR_INVALID, "MMSE system is not positive definite");
    for (int p = 0; p < n; ++p) {
      std::memcpy(J + (size_t)p * n, Jp.data() + (size_t)p * np, n * sizeof(double));
      h[p] = hp[p];
    }
    std::memcpy(xm, xp.data(), 2 * nt * sizeof(double));
    *n_out = n;
    return PIM_OK;
  } catch (...) {
    return fail(PIM_ERR_INVALID, "internal error in pim_mimo_ising_device");
  }
}
