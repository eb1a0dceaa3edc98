// MIMO detection as an Ising problem, built on the device in binary64.
//
// The same mapping as the host's pim_mimo_ising (Suppl. "MIMO problem
// definition", "Real-Valued equivalent", "Delta-Ising MIMO (DI-MIMO)
// formulation", "Baseline: linear MMSE detector"), one workgroup per request:
//
//   Hr = [[Re H, -Im H], [Im H, Re H]] (2Nr x 2Nt),  yr = [Re y; Im y],
//   G  = Hr^T Hr,
//   x_m = 0 (ML) or slice((G + I / esn0)^-1 Hr^T yr) (DI; LDL^T solve),
//   r  = yr - Hr x_m,  c = Hr^T r,
//   J  = -2 w_a w_b G_ij off the diagonal (spin a*2Nt + i carries weight w_a
//        on real component i),  h = 2 w_a c_i.
//
// Hr is never formed: its entries are read from the complex H (interleaved
// (re, im), row-major Nr x Nt), which is staged in LDS when it fits beside the
// lower triangle of G.  Every sum runs over its index in ascending order with
// separate multiplies and adds, as the host function does; the LDL^T factor
// is formed right-looking, which applies each element's subtractions in that
// same order, and the solves take the host's order too, so G, J, the factor
// and the unsliced MMSE estimate equal the host's bit for bit.  The triangular
// solves run in one wave (lane l owns rows l and l + 64).
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstring>
#include <type_traits>
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

// v of lane `lane` (the same in every lane of the wave) in every lane
__device__ __forceinline__ double bcast(double v, int lane) {
  const uint64_t b = (uint64_t)__double_as_longlong(v);
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)b, lane);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(b >> 32), lane);
  return __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
}

constexpr int kPanel = 8;  // LDL^T columns factored per panel

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

  // LDS: [H, y (staged)] | G lower triangle | z [n2] | x_m [n2] | r [m] | c [n2] |
  //      W of the factor's current panel [n2][kPanel] (DI)
  const int hy_len = STAGE_H ? 2 * nr * nt + 2 * nr : 0;
  double* G = smem + hy_len;
  double* z = G + n2 * (n2 + 1) / 2;
  double* xm = z + n2;
  double* r = xm + n2;
  double* c = r + m;
  double* Wp = c + n2;
  if (STAGE_H)
    for (int i = tid; i < hy_len; i += kThreads) smem[i] = Hg[i];
  if (tid == 0) bad = 0;
  __syncthreads();
  const double* Hs = STAGE_H ? smem : Hg;
  const double* ys = Hs + 2 * nr * nt;

  // ---- G = Hr^T Hr, lower triangle: thread (bi, bj) of an nb4 x nb4 grid
  //      takes rows i = bi + nb4 a and columns j = bj + nb4 b (a, b < 4), the
  //      entries with a >= b (the others lie above the diagonal), so that the
  //      lanes of a wave read consecutive columns of H; every entry summed
  //      over k in ascending order as above ----
  {
    const int nb4 = (n2 + 3) / 4;
    for (int t = tid; t < nb4 * nb4; t += kThreads) {
      const int bi = t / nb4, bj = t - bi * nb4;
      HrCol ci[4], cj[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        ci[q] = hr_col(nt, min(bi + nb4 * q, n2 - 1));
        cj[q] = hr_col(nt, min(bj + nb4 * q, n2 - 1));
      }
      double acc[4][4];
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b <= a; ++b) acc[a][b] = 0.0;
      for (int k = 0; k < nr; ++k) {  // rows k < nr of Hr
        const double* row = Hs + 2 * k * nt;
        double x[4], y[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          x[q] = ci[q].sg_lo * row[ci[q].off_lo];
          y[q] = cj[q].sg_lo * row[cj[q].off_lo];
        }
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
          for (int b = 0; b <= a; ++b) acc[a][b] += x[a] * y[b];
      }
      for (int k = 0; k < nr; ++k) {  // rows k >= nr
        const double* row = Hs + 2 * k * nt;
        double x[4], y[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          x[q] = ci[q].sg_hi * row[ci[q].off_hi];
          y[q] = cj[q].sg_hi * row[cj[q].off_hi];
        }
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
          for (int b = 0; b <= a; ++b) acc[a][b] += x[a] * y[b];
      }
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b <= a; ++b) {
          const int i = bi + nb4 * a, j = bj + nb4 * b;
          if (i < n2 && j <= i) G[tri(i, j)] = acc[a][b];
        }
    }
  }
  __syncthreads();
  // ---- J from G (zero diagonal, zero padding to npad x npad): a wave per
  //      row; spin p is component p - n2 of block 1 when p >= n2 (n <= 2 n2) ----
  for (int p = tid >> 6; p < a.npad; p += kThreads / 64) {
    const int pa = p >= n2 ? 1 : 0, i = p - pa * n2;
    double* Jrow = J + (size_t)p * a.npad;
    for (int q = tid & 63; q < a.npad; q += 64) {
      double v = 0.0;
      if (p < n && q < n && p != q) {
        const int qb = q >= n2 ? 1 : 0, j = q - qb * n2;
        v = -2.0 * (pa ? w1 : w0) * (qb ? w1 : w0) * G[i >= j ? tri(i, j) : tri(j, i)];
      }
      Jrow[q] = v;
    }
  }
  // ---- x_m ----
  if (map == PIM_MIMO_DI) {
    for (int i = tid; i < n2; i += kThreads) {  // b = Hr^T yr
      const HrCol a = hr_col(nt, i);
      double v = 0.0;
#pragma unroll 8
      for (int k = 0; k < nr; ++k) v += (a.sg_lo * Hs[2 * k * nt + a.off_lo]) * ys[2 * k];
#pragma unroll 8
      for (int k = 0; k < nr; ++k) v += (a.sg_hi * Hs[2 * k * nt + a.off_hi]) * ys[2 * k + 1];
      z[i] = v;
    }
    __syncthreads();  // J has read G: it becomes A = G + I / esn0, factored in place
    for (int i = tid; i < n2; i += kThreads) G[tri(i, i)] += 1.0 / rec.esn0;
    __syncthreads();
    // A = L D L^T (unit lower L, diagonal D) in panels of kPanel columns:
    //   W_ij = A_ij - sum_{l<j} W_il L_jl,  D_j = W_jj,  L_ij = W_ij / D_j.
    // (1) Wave 0 factors the panel: lane l holds rows j0 + l and j0 + l + 64
    // of the panel's columns in registers; per column every lane reads D_j
    // from its lane, the rows below are divided by it (W kept for the
    // updates) and W_il L_jl is subtracted from the later panel columns.
    // (2) All threads subtract W_ij L_kj of the panel's columns, in ascending
    // order, from the trailing matrix (rows and columns past the panel).
    // Each element thus receives its subtractions in ascending column order
    // and then its division, as in the host's column-by-column factorization.
    // The triangle ends with L below the diagonal and D on it.  A pivot that
    // is not positive (A not positive definite in binary64) marks the request
    // as failed.
    const int tr = tid >> 5, tc = tid & 31;
    for (int j0 = 0; j0 < n2; j0 += kPanel) {
      const int w = min(kPanel, n2 - j0);
      // fully unrolled over the panel's columns (register arrays indexed by
      // constants); FULL: w == kPanel, TWO: rows past j0 + 64 exist (both
      // uniform), so the common panels run without branches
      auto panel = [&](auto full_c, auto two_c) __attribute__((always_inline)) {
        constexpr bool FULL = decltype(full_c)::value, TWO = decltype(two_c)::value;
        constexpr int NQ = TWO ? 2 : 1;
        double P[NQ][kPanel];
        bool not_pd = false;
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
          const int r = tid + 64 * q, i = j0 + r;
#pragma unroll
          for (int c = 0; c < kPanel; ++c)
            P[q][c] = (i < n2 && (FULL || c < w) && c <= r) ? G[tri(i, j0 + c)] : 0.0;
        }
#pragma unroll
        for (int c = 0; c < kPanel; ++c) {
          if (FULL || c < w) {
            double d = bcast(P[0][c], c);  // row j0 + c is lane c
            not_pd = not_pd || !(d > 0.0);
            d = d > 0.0 ? d : 1.0;
            double Wv[NQ];
#pragma unroll
            for (int q = 0; q < NQ; ++q) {
              const int r = tid + 64 * q;
              Wv[q] = P[q][c];
              const double l = Wv[q] / d;
              P[q][c] = (r > c) ? l : Wv[q];
              if (j0 + r < n2) Wp[(j0 + r) * kPanel + c] = Wv[q];
            }
#pragma unroll
            for (int c2 = c + 1; c2 < kPanel; ++c2) {
              if (FULL || c2 < w) {
                const double lk = bcast(P[0][c], c2);  // L of row j0 + c2, column j0 + c
#pragma unroll
                for (int q = 0; q < NQ; ++q) {
                  const int r = tid + 64 * q;
                  const double u = P[q][c2] - Wv[q] * lk;
                  P[q][c2] = (r >= c2) ? u : P[q][c2];
                }
              }
            }
          }
        }
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
          const int r = tid + 64 * q, i = j0 + r;
#pragma unroll
          for (int c = 0; c < kPanel; ++c)
            if (i < n2 && (FULL || c < w) && c <= r) G[tri(i, j0 + c)] = P[q][c];
        }
        if (not_pd && tid == 0) bad = 1;
      };
      if (tid < 64) {
        using T = std::true_type;
        using F = std::false_type;
        const bool two = j0 + 64 < n2;
        if (w == kPanel) {
          if (two) panel(T{}, T{});
          else panel(T{}, F{});
        } else {
          if (two) panel(F{}, T{});
          else panel(F{}, F{});
        }
      }
      __syncthreads();
      const int b0 = j0 + w;  // trailing matrix: rows and columns >= b0 (fewer than 128)
      if (b0 < n2) {
        // this thread's rows i = b0 + tr + 32 qa and columns k = b0 + tc + 32 qb (k <= i)
        double lk[4][kPanel];
#pragma unroll
        for (int qb = 0; qb < 4; ++qb) {
          const int k = b0 + tc + 32 * qb;
#pragma unroll
          for (int c = 0; c < kPanel; ++c) lk[qb][c] = (k < n2 && c < w) ? G[tri(k, j0 + c)] : 0.0;
        }
#pragma unroll
        for (int qa = 0; qa < 4; ++qa) {
          const int i = b0 + tr + 32 * qa;
          if (i < n2) {
            double wi[kPanel];
#pragma unroll
            for (int c = 0; c < kPanel; ++c) wi[c] = c < w ? Wp[i * kPanel + c] : 0.0;
#pragma unroll
            for (int qb = 0; qb <= qa; ++qb) {
              const int k = b0 + tc + 32 * qb;
              if (k <= i) {
                double v = G[tri(i, k)];
#pragma unroll
                for (int c = 0; c < kPanel; ++c)
                  if (c < w) v = v - wi[c] * lk[qb][c];
                G[tri(i, k)] = v;
              }
            }
          }
        }
      }
      __syncthreads();
    }
    // L w = b, y = w / D, then L^T z = y, in wave 0: lane l owns rows l and
    // l + 64.  Step k broadcasts the final value of row k from its lane, the
    // owner keeps it, and every lane subtracts its row's term; rows that are
    // already final, or past n2, take a don't-care term (they are never read
    // again), and the step count is rounded up to a multiple of kAhead with
    // such don't-care steps, which keeps the steps free of branches.  The
    // factor entries are loaded kAhead steps before they are used.  Row i
    // takes its subtractions in ascending k going forward and descending k
    // going back, as the host's solve does.
    if (tid < 64) {
      constexpr int kAhead = 4;
      const int last = n2 - 1, steps = (n2 + kAhead - 1) / kAhead * kAhead;
      // L_ik for i > k, and some finite entry of the triangle otherwise
      auto l_row = [&](int i, int k) {
        const int ii = max(min(i, last), 0), kk = max(min(k, ii), 0);
        return G[tri(ii, kk)];
      };
      double zr[2], zf[2], dg[2], lb[kAhead][2];
#pragma unroll
      for (int q = 0; q < 2; ++q) {
        const int i = tid + 64 * q;
        zr[q] = i < n2 ? z[i] : 0.0;
        zf[q] = 0.0;
        dg[q] = i < n2 ? G[tri(i, i)] : 1.0;
      }
#pragma unroll
      for (int s = 0; s < kAhead; ++s)
#pragma unroll
        for (int q = 0; q < 2; ++q) lb[s][q] = l_row(tid + 64 * q, s);
      for (int k0 = 0; k0 < steps; k0 += kAhead) {  // forward
#pragma unroll
        for (int s = 0; s < kAhead; ++s) {
          const int k = k0 + s;
          const double z0 = bcast(zr[0], k & 63), z1 = bcast(zr[1], k & 63);
          const double zk = k < 64 ? z0 : z1;
#pragma unroll
          for (int q = 0; q < 2; ++q) {
            zf[q] = tid + 64 * q == k ? zk : zf[q];
            zr[q] = zr[q] - lb[s][q] * zk;
            lb[s][q] = l_row(tid + 64 * q, k + kAhead);
          }
          __builtin_amdgcn_sched_barrier(0);  // keeps the loads in this step, kAhead steps before their use
        }
      }
#pragma unroll
      for (int q = 0; q < 2; ++q) {
        zr[q] = zf[q] / dg[q];
        zf[q] = 0.0;
      }
#pragma unroll
      for (int s = 0; s < kAhead; ++s)
#pragma unroll
        for (int q = 0; q < 2; ++q) lb[s][q] = l_row(last - s, tid + 64 * q);
      for (int k0 = last; k0 > last - steps; k0 -= kAhead) {  // backward: L_ki for i < k
#pragma unroll
        for (int s = 0; s < kAhead; ++s) {
          const int k = k0 - s;
          const double z0 = bcast(zr[0], k & 63), z1 = bcast(zr[1], k & 63);
          const double zk = k < 64 ? z0 : z1;
#pragma unroll
          for (int q = 0; q < 2; ++q) {
            zf[q] = tid + 64 * q == k ? zk : zf[q];
            zr[q] = zr[q] - lb[s][q] * zk;
            lb[s][q] = l_row(k - kAhead, tid + 64 * q);
          }
          __builtin_amdgcn_sched_barrier(0);
        }
      }
#pragma unroll
      for (int q = 0; q < 2; ++q)
        if (tid + 64 * q < n2) z[tid + 64 * q] = zf[q];
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
#pragma unroll 8
    for (int j = 0; j < n2; ++j) v -= hr_at(Hs, nr, nt, k, j) * xm[j];
    r[k] = v;
  }
  __syncthreads();
  for (int i = tid; i < n2; i += kThreads) {
    const HrCol a = hr_col(nt, i);
    double v = 0.0;
#pragma unroll 8
    for (int k = 0; k < nr; ++k) v += (a.sg_lo * Hs[2 * k * nt + a.off_lo]) * r[k];
#pragma unroll 8
    for (int k = 0; k < nr; ++k) v += (a.sg_hi * Hs[2 * k * nt + a.off_hi]) * r[nr + k];
    c[i] = v;
  }
  __syncthreads();
  for (int p = tid; p < a.npad; p += kThreads) hv[p] = p < n ? 2.0 * ((p / n2) ? w1 : w0) * c[p % n2] : 0.0;
  for (int i = tid; i < a.xm_stride; i += kThreads) xm_out[i] = i < n2 ? xm[i] : 0.0;
}

}  // namespace

size_t mimo_map_work_doubles(int nr, int nt) {
  // LDS doubles of one request besides its staged H and y: G triangle, z, x_m,
  // r, c and the factor's panel W
  const size_t n2 = 2 * (size_t)nt, m = 2 * (size_t)nr;
  return n2 * (n2 + 1) / 2 + 3 * n2 + m + n2 * kPanel;
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
