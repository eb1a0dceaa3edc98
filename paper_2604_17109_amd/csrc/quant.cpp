// Host quantisation of real-valued couplings into the MFMA operand formats.
//
// FP8 is OCP e4m3 ("fn": exponent bias 7, three mantissa bits, no infinities,
// largest finite value 448 = 0x7E); BF16 is the top half of binary32.  Both
// round to nearest with ties to even, directly from binary64 (no double
// rounding through binary32), and FP8 saturates at +-448.
#include <cmath>
#include <cstdint>
#include <cstring>

#include "internal.hpp"

namespace pim {
namespace {

// Exponent field of a binary64 value minus its bias: E with x in [2^E, 2^(E+1))
// for normal x (-1023 for zero and subnormals).
int exponent_of(double x) {
  uint64_t u;
  std::memcpy(&u, &x, sizeof u);
  return (int)((u >> 52) & 0x7FF) - 1023;
}

// 2^k as a binary64 value, -1022 <= k <= 1023 (exact).
double pow2(int k) {
  const uint64_t u = (uint64_t)(k + 1023) << 52;
  double x;
  std::memcpy(&x, &u, sizeof x);
  return x;
}

// Round to the nearest integer, ties to even, for 0 <= v <= 2^52: adding 2^52
// leaves no fraction bits, so the addition itself rounds (binary64, default
// rounding mode) and the subtraction is exact.
double rint_small(double v) {
  const double big = 4503599627370496.0;  // 2^52
  volatile double t = v + big;            // kept as written: not folded to v
  return t - big;
}

}  // namespace

uint8_t fp8_e4m3_rne(double x) {
  if (x == 0.0 || std::isnan(x)) return 0;
  const uint8_t sign = x < 0.0 ? 0x80 : 0x00;
  const double a = std::fabs(x);
  if (a >= 448.0) return sign | 0x7E;
  if (a < 0.015625) {                               // below 2^-6: subnormal steps of 2^-9
    const double q = rint_small(a * 512.0);         // exact scaling, ties to even; q in [0, 8]
    return sign | (uint8_t)q;                       // q = 8 is the smallest normal, code 0x08
  }
  int E = exponent_of(a);                           // a in [2^E, 2^(E+1)), -6 <= E <= 8
  double q = rint_small(a * pow2(3 - E));           // significand x 8, in [8, 16]
  if (q == 16.0) {
    q = 8.0;
    ++E;
  }
  if (E > 8 || (E == 8 && q > 14.0)) return sign | 0x7E;
  return sign | (uint8_t)(((E + 7) << 3) | ((int)q - 8));
}

double fp8_e4m3_value(uint8_t c) {
  const double sign = (c & 0x80) ? -1.0 : 1.0;
  const int ex = (c >> 3) & 0xF, m = c & 7;
  if (ex == 0) return sign * (double)m * pow2(-9);
  return sign * (8.0 + m) * pow2(ex - 10);
}

uint16_t bf16_rne(double x) {
  if (x == 0.0 || std::isnan(x)) return 0;
  const uint16_t sign = x < 0.0 ? 0x8000 : 0x0000;
  if (std::isinf(x)) return sign | 0x7F80;
  const double a = std::fabs(x);
  int E = exponent_of(a);                            // a in [2^E, 2^(E+1)) (-1023: subnormal a)
  if (E < -126) {                                    // subnormal: steps of 2^-133
    const double q = rint_small(a * pow2(133));      // a < 2^-126: exact, q in [0, 128]
    return sign | (uint16_t)q;                       // q = 128 is the smallest normal
  }
  double q = rint_small(a * pow2(7 - E));            // significand x 128, in [128, 256]
  if (q == 256.0) {
    q = 128.0;
    ++E;
  }
  if (E > 127) return sign | 0x7F80;
  return sign | (uint16_t)(((E + 127) << 7) | ((int)q - 128));
}

double bf16_value(uint16_t c) {
  const double sign = (c & 0x8000) ? -1.0 : 1.0;
  const int ex = (c >> 7) & 0xFF, m = c & 0x7F;
  if (ex == 0) return sign * (double)m * pow2(-133);
  if (ex == 0xFF) return sign * INFINITY;
  return sign * (128.0 + m) * pow2(ex - 134);
}

float real_scale(const double* J, size_t count, int prec) {
  double m = 0.0;
  for (size_t i = 0; i < count; ++i) m = std::fmax(m, std::fabs(J[i]));
  if (m == 0.0) return 1.0f;
  if (prec == PIM_PREC_FP8) return (float)(m / 448.0);
  int e;
  (void)std::frexp(m, &e);
  return (float)std::ldexp(1.0, e - 1);              // power of two: max |J| / scale in [1, 2)
}

double quantized_value(double x, int prec, float scale) {
  const double y = x / (double)scale;
  return prec == PIM_PREC_FP8 ? fp8_e4m3_value(fp8_e4m3_rne(y)) : bf16_value(bf16_rne(y));
}

}  // namespace pim
