// Host schedule compiler: turns the binary64 update rule of one step into
// integer thresholds on the exact integer field I and the B-bit noise index u.
//
// The rule (Eq. (4); LUT from Suppl. "Quantization scheme", Algorithm
// "LUT-based tanh approximation"), with every real operation in IEEE binary64
// round-to-nearest in the order written:
//   g   = beta * c
//   x   = g * I                                  (I an exact integer)
//   k   = #{ j in 1..L-1 : x >= b_j },  b_j = (2j - L) / L
//   a   = lev_k + (s > 0 ? xi : -xi),   lev_k = (2k - (L-1)) / (L-1)
//   w   = eta * Z[u]
//   v   = a + w;  s' = +1 if v > 0, -1 if v < 0, s if v == 0.
// Because v == 0 exactly when w == -a, s' = +1 <=> (s > 0 ? w >= -a : w > -a).
// Rounding is monotone, so x is non-decreasing in I and w non-decreasing in u:
// each comparison becomes one integer threshold.
//
// This file is compiled with -ffp-contract=off: no fused multiply-add may
// change a rounding.
#include <cfloat>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <vector>

#include "internal.hpp"

namespace pim {
namespace {

constexpr int32_t kThetaLo = -32768;  // every |I| <= kFieldLimit satisfies I >= this
constexpr int32_t kThetaHi = 32767;   // no |I| <= kFieldLimit satisfies I >= this

double breakpoint(int j, int L) { return (double)(2 * j - L) / (double)L; }
double level(int k, int L) { return (double)(2 * k - (L - 1)) / (double)(L - 1); }

// Smallest integer I with fl(g * I) >= b, clamped to [kThetaLo, kThetaHi].
int32_t field_threshold(double g, double b) {
  if (g == 0.0) {
    // fl(0 * I) is +-0 for every I, and (+-0 >= b) <=> (0 >= b).
    return (0.0 >= b) ? kThetaLo : kThetaHi;
  }
  const double q0 = std::ceil(b / g);
  if (!(q0 > -40000.0)) return kThetaLo;
  if (!(q0 < 40000.0)) return kThetaHi;
  int64_t q = (int64_t)q0;
  // fl(g * I) is non-decreasing in I; step to the exact boundary.
  while (g * (double)(q - 1) >= b) --q;
  while (g * (double)q < b) ++q;
  if (q < kThetaLo) return kThetaLo;
  if (q > kThetaHi) return kThetaHi;
  return (int32_t)q;
}

}  // namespace

// umin[2k + (s<0)]: smallest u with s(t+1) = +1 in LUT bin k (2^B if none).
void compile_umin(const Rule& r, double eta, int32_t* umin) {
  const int L = r.levels;
  const int nu = (int)r.ztab.size();
  for (int k = 0; k < L; ++k) {
    for (int sneg = 0; sneg < 2; ++sneg) {
      const double a = level(k, L) + (sneg ? -r.xi : r.xi);
      const double neg_a = -a;
      // predicate is monotone in u: binary search for the first u where it holds
      int lo = 0, hi = nu;  // answer in [lo, hi]
      while (lo < hi) {
        const int mid = (lo + hi) / 2;
        const double w = eta * r.ztab[mid];
        const bool up = sneg ? (w > neg_a) : (w >= neg_a);
        if (up) hi = mid; else lo = mid + 1;
      }
      umin[2 * k + sneg] = lo;
    }
  }
}

void compile_step(const Rule& r, double beta, double eta, int32_t* theta, int32_t* umin) {
  const int L = r.levels;
  const double g = beta * r.c;
  for (int j = 1; j < L; ++j) theta[j - 1] = field_threshold(g, breakpoint(j, L));
  compile_umin(r, eta, umin);
}

namespace {
// Total order of the floats as unsigned keys: -inf < ... < -0 < +0 < ... < +inf.
uint32_t float_key(float f) {
  uint32_t b;
  std::memcpy(&b, &f, 4);
  return (b & 0x80000000u) ? ~b : (b | 0x80000000u);
}
float key_float(uint32_t k) {
  const uint32_t b = (k & 0x80000000u) ? (k & 0x7FFFFFFFu) : ~k;
  float f;
  std::memcpy(&f, &b, 4);
  return f;
}

// Smallest float x with fl(g * x) >= b (x converted to binary64 exactly):
// -inf when every finite x qualifies, +inf when none does.  fl(g * x) is
// non-decreasing in x for g >= 0, so the predicate is monotone over the key
// order and a bisection over the 2^32 keys finds the boundary.  -0 and +0
// share the predicate's value, so the result is never +0.
float field_threshold_real(double g, double b) {
  auto ok = [&](float x) { return g * (double)x >= b; };
  if (ok(-FLT_MAX)) return -INFINITY;
  if (!ok(FLT_MAX)) return INFINITY;
  uint32_t lo = float_key(-FLT_MAX), hi = float_key(FLT_MAX);  // ok(lo) false, ok(hi) true
  while (hi - lo > 1) {
    const uint32_t mid = lo + (hi - lo) / 2;
    if (ok(key_float(mid))) hi = mid; else lo = mid;
  }
  return key_float(hi);
}
}  // namespace

void compile_step_real(const Rule& r, double beta, double eta, float* theta, int32_t* umin) {
  const int L = r.levels;
  const double g = beta * r.c;
  for (int j = 1; j < L; ++j) theta[j - 1] = field_threshold_real(g, breakpoint(j, L));
  compile_umin(r, eta, umin);
}

void theta_by_noise_real(const float* theta, const int32_t* umin, int levels, float* tab) {
  // as theta_by_noise, over float fields, with index u for s = +1 and ~u for
  // s = -1 relative to the centre kNoiseVals
  for (int sneg = 0; sneg < 2; ++sneg) {
    for (int m = 0; m <= levels; ++m) {
      const int lo = (m == levels) ? 0 : umin[2 * m + sneg];
      const int hi = (m == 0) ? kNoiseVals : umin[2 * (m - 1) + sneg];
      float th;
      if (m == 0) th = -INFINITY;
      else if (m >= levels) th = INFINITY;
      else th = theta[m - 1];
      for (int u = lo; u < hi; ++u) tab[kNoiseVals + (sneg ? ~u : u)] = th;
    }
  }
}

void theta_by_noise(const int32_t* theta, const int32_t* umin, int levels, int16_t* tab) {
  // s' = +1 <=> bin(I) >= kmin(u, s), with kmin = #{k : u < umin[k][s]}
  // (umin is non-increasing in k), and bin(I) >= m <=> I >= theta_m.  So kmin
  // is constant on the u-ranges [umin[k][s], umin[k-1][s]): fill them.
  for (int sneg = 0; sneg < 2; ++sneg) {
    for (int m = 0; m <= levels; ++m) {
      // u-range with kmin == m: u >= umin[m][s] (or 0 when m == L) and
      // u < umin[m-1][s] (or 2^B when m == 0)
      const int lo = (m == levels) ? 0 : umin[2 * m + sneg];
      const int hi = (m == 0) ? kNoiseVals : umin[2 * (m - 1) + sneg];
      int32_t th;
      if (m == 0) th = kThetaLo;
      else if (m >= levels) th = kThetaHi;
      else th = theta[m - 1];
      for (int u = lo; u < hi; ++u) {
        // index relative to the centre kNoiseVals: u ^ s with s = +-1 as int
        const int idx = sneg ? ~u : (u ^ 1);
        tab[kNoiseVals + idx] = (int16_t)th;
      }
    }
  }
}

namespace {
// Standard normal CDF through the C library's erfc.
double normal_cdf(double x) { return 0.5 * std::erfc(-x / std::sqrt(2.0)); }
double normal_pdf(double x) { return std::exp(-0.5 * x * x) / std::sqrt(2.0 * M_PI); }

// Quantile by bisection on [-40, 40] followed by Newton polishing.
double normal_quantile(double p) {
  double lo = -40.0, hi = 40.0;
  for (int i = 0; i < 200 && hi - lo > 1e-15; ++i) {
    const double mid = 0.5 * (lo + hi);
    if (normal_cdf(mid) < p) lo = mid; else hi = mid;
  }
  double x = 0.5 * (lo + hi);
  for (int i = 0; i < 3; ++i) {
    const double d = normal_pdf(x);
    if (d <= 0) break;
    x -= (normal_cdf(x) - p) / d;
  }
  return x;
}
}  // namespace

bool builtin_noise_table(int noise, std::vector<double>& out) {
  out.assign(kNoiseVals, 0.0);
  const double m = (double)kNoiseVals;
  if (noise == PIM_NOISE_UNIFORM) {
    for (int u = 0; u < kNoiseVals; ++u) out[u] = (2.0 * u + 1.0 - m) / m;
    return true;
  }
  if (noise == PIM_NOISE_GAUSS) {
    for (int u = 0; u < kNoiseVals / 2; ++u) {
      const double z = normal_quantile((u + 0.5) / m);
      out[u] = z;
      out[kNoiseVals - 1 - u] = -z;  // exact odd symmetry of the midpoints
    }
    return true;
  }
  return false;
}

}  // namespace pim
