// MIMO detection as an Ising problem (host, binary64).
//
// Suppl. "MIMO problem definition": y = H x + n with complex H [Nr x Nt].  The
// real-valued equivalent stacks real and imaginary parts:
//     Hr = [[Re H, -Im H], [Im H, Re H]]  (2Nr x 2Nt),  yr = [Re y; Im y].
// Suppl. "Delta-Ising MIMO (DI-MIMO) formulation": with x = x_m + T s,
// s in {-1, +1}^K, the residual ||yr - Hr (x_m + T s)||^2 equals, up to a
// constant, -h^T s - s^T J_DI s with J_DI = -zeroDiag(T^T Hr^T Hr T) and
// h = 2 T^T Hr^T (yr - Hr x_m).  The library's instances follow Eq. (1), which
// counts each pair once, so the couplings handed out are J = 2 J_DI.
//
// Two mappings: ML (x_m = 0, T = I for 4-QAM and [2I, I] for 16-QAM, so T s
// covers the constellation exactly) and DI (x_m = the MMSE estimate of Suppl.
// "Baseline: linear MMSE detector", sliced to the constellation, T = [I, I]).
// Slicing maps v to the odd integer 2 floor(v / 2) + 1, clipped to the
// constellation's levels.
#include <cmath>
#include <cstdint>
#include <cstring>
#include <vector>

#include "internal.hpp"

namespace pim {
namespace {

int pam_half(int qam) { return qam == 4 ? 1 : 3; }  // largest level per real component

double slice_level(double v, int qam) {
  const double m = pam_half(qam);
  const double q = 2.0 * std::floor(v / 2.0) + 1.0;
  return q < -m ? -m : (q > m ? m : q);
}

// T = [w_0 I, w_1 I, ...]: block weights of the mapping.
int transform_weights(int qam, int map, double* w) {
  if (map == PIM_MIMO_ML) {
    if (qam == 4) {
      w[0] = 1.0;
      return 1;
    }
    w[0] = 2.0;
    w[1] = 1.0;
    return 2;
  }
  w[0] = 1.0;
  w[1] = 1.0;
  return 2;
}

// Real-valued equivalent of the complex model.
void real_model(const double* Hc, const double* yc, int nr, int nt, std::vector<double>& H, std::vector<double>& y) {
  const int m = 2 * nr, n = 2 * nt;
  H.assign((size_t)m * n, 0.0);
  y.assign(m, 0.0);
  for (int i = 0; i < nr; ++i) {
    for (int j = 0; j < nt; ++j) {
      const double re = Hc[2 * ((size_t)i * nt + j)], im = Hc[2 * ((size_t)i * nt + j) + 1];
      H[(size_t)i * n + j] = re;
      H[(size_t)i * n + nt + j] = -im;
      H[(size_t)(nr + i) * n + j] = im;
      H[(size_t)(nr + i) * n + nt + j] = re;
    }
    y[i] = yc[2 * i];
    y[nr + i] = yc[2 * i + 1];
  }
}

// Solves A z = b for symmetric positive definite A (n x n) by an LDL^T
// factorization (unit lower L, diagonal D, no square roots):
//   W_ij = A_ij - sum_{l<j} W_il L_jl (l ascending, i >= j),  D_j = W_jj,
//   L_ij = W_ij / D_j (i > j),
// then L w = b, y = w / D and L^T z = y, each row's subtractions taken in
// ascending k going forward and from the last row's term back going back.
// The device mapping (mimo_map.hip) performs the same operations in the same
// order, so both give the same z bit for bit.
bool spd_solve(const std::vector<double>& A, const std::vector<double>& b, int n, std::vector<double>& z) {
  std::vector<double> W((size_t)n * n, 0.0), L((size_t)n * n, 0.0), D(n);
  for (int j = 0; j < n; ++j) {
    for (int i = j; i < n; ++i) {
      double v = A[(size_t)i * n + j];
      for (int l = 0; l < j; ++l) v -= W[(size_t)i * n + l] * L[(size_t)j * n + l];
      W[(size_t)i * n + j] = v;
    }
    D[j] = W[(size_t)j * n + j];
    if (!(D[j] > 0.0)) return false;
    for (int i = j + 1; i < n; ++i) L[(size_t)i * n + j] = W[(size_t)i * n + j] / D[j];
  }
  z = b;
  for (int i = 0; i < n; ++i) {  // L w = b
    double v = z[i];
    for (int k = 0; k < i; ++k) v -= L[(size_t)i * n + k] * z[k];
    z[i] = v;
  }
  for (int i = 0; i < n; ++i) z[i] = z[i] / D[i];
  for (int i = n - 1; i >= 0; --i) {  // L^T z = y
    double v = z[i];
    for (int k = n - 1; k > i; --k) v -= L[(size_t)k * n + i] * z[k];
    z[i] = v;
  }
  return true;
}

}  // namespace
}  // namespace pim

using namespace pim;

extern "C" {

pim_status pim_mimo_ising(const double* Hc, const double* yc, int32_t nr, int32_t nt, int32_t qam, int32_t map,
                          double esn0, double* J, double* h, double* xm, int32_t* n_out) {
  try {
    if (!Hc || !yc || !J || !h || !xm || !n_out) return fail(PIM_ERR_INVALID, "NULL argument");
    if (nr < 1 || nt < 1 || 4 * nt > PIM_MAX_N_LDS)
      return fail(PIM_ERR_INVALID, "nr = %d, nt = %d: need nr, nt >= 1 and 4 nt <= %d", nr, nt, PIM_MAX_N_LDS);
    if (qam != 4 && qam != 16) return fail(PIM_ERR_UNSUPPORTED, "qam = %d (4 and 16 are implemented)", qam);
    if (map != PIM_MIMO_ML && map != PIM_MIMO_DI) return fail(PIM_ERR_INVALID, "unknown mapping %d", map);
    if (map == PIM_MIMO_DI && !(std::isfinite(esn0) && esn0 > 0.0))
      return fail(PIM_ERR_INVALID, "esn0 must be finite and > 0 for the DI mapping");
    for (int i = 0; i < 2 * nr * nt; ++i)
      if (!std::isfinite(Hc[i])) return fail(PIM_ERR_INVALID, "H is not finite");
    for (int i = 0; i < 2 * nr; ++i)
      if (!std::isfinite(yc[i])) return fail(PIM_ERR_INVALID, "y is not finite");
    const int m = 2 * nr, n2 = 2 * nt;
    std::vector<double> H, y;
    real_model(Hc, yc, nr, nt, H, y);
    std::vector<double> x0(n2, 0.0);
    if (map == PIM_MIMO_DI) {
      // MMSE: (Hr^T Hr + I / esn0) z = Hr^T yr, the real form of the complex filter
      std::vector<double> A((size_t)n2 * n2), b(n2), z;
      for (int i = 0; i < n2; ++i) {
        for (int j = 0; j < n2; ++j) {
          double v = 0.0;
          for (int k = 0; k < m; ++k) v += H[(size_t)k * n2 + i] * H[(size_t)k * n2 + j];
          A[(size_t)i * n2 + j] = v;
        }
        A[(size_t)i * n2 + i] += 1.0 / esn0;
        double v = 0.0;
        for (int k = 0; k < m; ++k) v += H[(size_t)k * n2 + i] * y[k];
        b[i] = v;
      }
      if (!spd_solve(A, b, n2, z)) return fail(PIM_ERR_INVALID, "MMSE system is not positive definite");
      for (int i = 0; i < n2; ++i) x0[i] = slice_level(z[i], qam);
    }
    double w[2];
    const int nb = transform_weights(qam, map, w);
    const int n = nb * n2;
    // G = Hr^T Hr (n2 x n2), c = Hr^T (yr - Hr x_m)
    std::vector<double> r(m), G((size_t)n2 * n2), c(n2);
    for (int k = 0; k < m; ++k) {
      double v = y[k];
      for (int j = 0; j < n2; ++j) v -= H[(size_t)k * n2 + j] * x0[j];
      r[k] = v;
    }
    for (int i = 0; i < n2; ++i) {
      for (int j = 0; j < n2; ++j) {
        double v = 0.0;
        for (int k = 0; k < m; ++k) v += H[(size_t)k * n2 + i] * H[(size_t)k * n2 + j];
        G[(size_t)i * n2 + j] = v;
      }
      double v = 0.0;
      for (int k = 0; k < m; ++k) v += H[(size_t)k * n2 + i] * r[k];
      c[i] = v;
    }
    // spin a*n2 + i carries weight w_a on real component i
    for (int a = 0; a < nb; ++a)
      for (int i = 0; i < n2; ++i) {
        const int p = a * n2 + i;
        h[p] = 2.0 * w[a] * c[i];
        for (int bb = 0; bb < nb; ++bb)
          for (int j = 0; j < n2; ++j) {
            const int q = bb * n2 + j;
            J[(size_t)p * n + q] = (p == q) ? 0.0 : -2.0 * w[a] * w[bb] * G[(size_t)i * n2 + j];
          }
      }
    std::memcpy(xm, x0.data(), n2 * sizeof(double));
    *n_out = n;
    return PIM_OK;
  } catch (...) {
    return fail(PIM_ERR_INVALID, "internal error in pim_mimo_ising");
  }
}

pim_status pim_mimo_decode(const double* xm, const int8_t* s, int32_t nt, int32_t qam, int32_t map, double* x) {
  if (!xm || !s || !x) return fail(PIM_ERR_INVALID, "NULL argument");
  if (nt < 1 || 4 * nt > PIM_MAX_N_LDS) return fail(PIM_ERR_INVALID, "nt = %d out of range", nt);
  if (qam != 4 && qam != 16) return fail(PIM_ERR_UNSUPPORTED, "qam = %d (4 and 16 are implemented)", qam);
  if (map != PIM_MIMO_ML && map != PIM_MIMO_DI) return fail(PIM_ERR_INVALID, "unknown mapping %d", map);
  double w[2];
  const int nb = transform_weights(qam, map, w);
  const int n2 = 2 * nt;
  for (int i = 0; i < n2; ++i) {
    double v = xm[i];
    for (int a = 0; a < nb; ++a) {
      const int8_t sv = s[a * n2 + i];
      if (sv != 1 && sv != -1) return fail(PIM_ERR_INVALID, "spin %d is not +-1", a * n2 + i);
      v += w[a] * sv;
    }
    const double q = slice_level(v, qam);
    // component i < nt is the real part of symbol i, i >= nt the imaginary part
    if (i < nt) x[2 * i] = q;
    else x[2 * (i - nt) + 1] = q;
  }
  return PIM_OK;
}

}  // extern "C"
