// Host quantisation of real-valued couplings into the MFMA operand formats.
//
// FP8 is OCP e4m3 ("fn": exponent bias 7, three mantissa bits, no infinities,
// largest finite value 448 = 0x7E); BF16 is the top half of binary32.  Both
// round to nearest with ties to even, directly from binary64 (no double
// rounding through binary32), and FP8 saturates at +-448.
#include <cmath>
#include <cstdint>

#include "internal.hpp"

namespace pim {

uint8_t fp8_e4m3_rne(double x) {
  if (x == 0.0 || std::isnan(x)) return 0;
  const uint8_t sign = x < 0.0 ? 0x80 : 0x00;
  const double a = std::fabs(x);
  if (a >= 448.0) return sign | 0x7E;
  if (a < 0.015625) {                               // below 2^-6: subnormal steps of 2^-9
    const double q = std::nearbyint(a * 512.0);     // exact scaling, ties to even; q in [0, 8]
    return sign | (uint8_t)q;                       // q = 8 is the smallest normal, code 0x08
  }
  int e;
  (void)std::frexp(a, &e);
  int E = e - 1;                                     // a in [2^E, 2^(E+1))
  double q = std::nearbyint(std::ldexp(a, 3 - E));   // significand x 8, in [8, 16]
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
  if (ex == 0) return sign * std::ldexp((double)m, -9);
  return sign * std::ldexp(8.0 + m, ex - 10);
}

uint16_t bf16_rne(double x) {
  if (x == 0.0 || std::isnan(x)) return 0;
  const uint16_t sign = x < 0.0 ? 0x8000 : 0x0000;
  if (std::isinf(x)) return sign | 0x7F80;
  const double a = std::fabs(x);
  int e;
  (void)std::frexp(a, &e);
  int E = e - 1;
  if (E < -126) {                                    // subnormal: steps of 2^-133
    const double q = std::nearbyint(std::ldexp(a, 133));
    return sign | (uint16_t)q;                       // q = 128 is the smallest normal
  }
  double q = std::nearbyint(std::ldexp(a, 7 - E));   // significand x 128, in [128, 256]
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
  if (ex == 0) return sign * std::ldexp((double)m, -133);
  if (ex == 0xFF) return sign * INFINITY;
  return sign * std::ldexp(128.0 + m, ex - 134);
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
