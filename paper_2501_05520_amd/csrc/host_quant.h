// Host-side weight quantisation for the FP8 mode (plain C++, no device code).
#pragma once
#include <stdint.h>
#include <stddef.h>

#include <algorithm>
#include <cmath>

// OCP FP8 E4M3 encoding (1 sign, 4 exponent bits with bias 7, 3 mantissa bits;
// largest finite 448, subnormal step 2^-9) with round-to-nearest-even and
// saturation to +-448.  Scaling by a power of two is exact, so the rounding is done
// on a / 2^(e-3), which is exact in float, with the current (nearest-even) mode.
inline uint8_t host_f2e4m3(float f) {
  const uint8_t sign = std::signbit(f) ? 0x80 : 0;
  const float a = std::fabs(f);
  if (std::isnan(f)) return 0x7f;
  if (a >= 448.f) return sign | 0x7e;
  int e2;
  std::frexp(a, &e2);              // a = m 2^e2, m in [0.5, 1)
  const int E = e2 - 1;            // a in [2^E, 2^(E+1))
  if (a == 0.f || E < -6) {        // subnormal: a = q 2^-9
    const int q = (int)std::nearbyint(std::ldexp(a, 9));   // 0..8; 8 carries into 2^-6
    return sign | (uint8_t)q;
  }
  int q = (int)std::nearbyint(std::ldexp(a, 3 - E));         // 8..16
  int Eb = E + 7;
  if (q == 16) { q = 8; ++Eb; }
  const int code = (Eb << 3) | (q - 8);
  return sign | (uint8_t)(code > 0x7e ? 0x7e : code);
}

// Per-tensor power-of-two scale s with max|w| * s <= 448 (s = 1 for a zero tensor).
inline float fp8_weight_scale(const float* w, size_t n) {
  float amax = 0.f;
  for (size_t i = 0; i < n; ++i) amax = std::max(amax, std::fabs(w[i]));
  if (!(amax > 0.f)) return 1.f;
  return std::ldexp(1.f, (int)std::floor(std::log2(448.0 / amax)));
}

