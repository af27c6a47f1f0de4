// Counter-based generator of the synthetic inputs, shared by the library's device kernels and
// its host code (and compiled on its own by a CPU test).  It is the twin of the Python module
// that feeds the oracle and must reproduce its values bit for bit:
//   * SplitMix64 output function (Steele, Lea & Flood, OOPSLA 2014) on the counter state
//     key(seed, stream) + (index + 1) * golden;
//   * uniforms (0, 1) from the top 53 bits;
//   * normals by Box-Muller (cosine branch) of uniforms 2i and 2i + 1;
//   * the logarithm, the cosine of a fraction of a turn and the exponential from exact range
//     reductions and truncated series with exact binary coefficients -- only IEEE +, -, *, /
//     and sqrt, each correctly rounded, evaluated in a fixed order with no contraction into
//     fused multiply-adds, so every platform produces the same bits.
// Value recipe of the workloads: eps_o ~ U[-1.5, -0.3], eps_v ~ U[0.1, 5.0] (each sorted),
// L^K_pq = gamma N(0,1) e^(-K/decay) (upper triangle drawn, mirrored), amplitude factors
// N(0,1)/sqrt(nP), ERI-grid factors N(0,1)/sqrt(nQ).
#pragma once
#include <stdint.h>

#if defined(__HIPCC__)
#define THC_HD __host__ __device__
#else
#define THC_HD
#endif
#if defined(__clang__)
#define THC_NOCONTRACT _Pragma("clang fp contract(off)")
#else
#define THC_NOCONTRACT
#endif

namespace thc_synth {

enum Stream : uint64_t { EPS_O = 0, EPS_V = 1, CHOL = 2, XO_AMP = 3, XV_AMP = 4, XO_ERI = 5, XV_ERI = 6 };

constexpr uint64_t GOLDEN = 0x9E3779B97F4A7C15ull;

THC_HD inline uint64_t mix(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

THC_HD inline uint64_t key(uint64_t seed, uint64_t stream) { return mix(seed * GOLDEN ^ mix(stream + GOLDEN)); }

THC_HD inline uint64_t bits(uint64_t k, uint64_t idx) { return mix(k + (idx + 1) * GOLDEN); }

THC_HD inline double from_bits(uint64_t b) {
  union {
    uint64_t u;
    double d;
  } x;
  x.u = b;
  return x.d;
}
THC_HD inline uint64_t to_bits(double d) {
  union {
    uint64_t u;
    double d;
  } x;
  x.d = d;
  return x.u;
}

THC_HD inline double uniform(uint64_t k, uint64_t idx) {
  THC_NOCONTRACT
  return ((double)(bits(k, idx) >> 11) + 0.5) * 0x1.0p-53;
}

// ln u for a normal u > 0: u = m 2^e with m in [sqrt(1/2), sqrt(2)), then
// e ln 2 + 2 atanh(s), s = (m - 1)/(m + 1), by 11 terms of its series.
THC_HD inline double gen_log(double u) {
  THC_NOCONTRACT
  const uint64_t b = to_bits(u);
  int e = (int)((b >> 52) & 0x7ff) - 1022;
  double m = from_bits((b & 0x800fffffffffffffull) | (uint64_t(1022) << 52));  // [0.5, 1)
  if (m < 0x1.6a09e667f3bcdp-1) {
    m = m * 2.0;
    e -= 1;
  }
  const double s = (m - 1.0) / (m + 1.0);
  const double s2 = s * s;
  double p = 0x1.8618618618618p-5;
  p = p * s2 + 0x1.af286bca1af28p-5;
  p = p * s2 + 0x1.e1e1e1e1e1e1ep-5;
  p = p * s2 + 0x1.1111111111111p-4;
  p = p * s2 + 0x1.3b13b13b13b14p-4;
  p = p * s2 + 0x1.745d1745d1746p-4;
  p = p * s2 + 0x1.c71c71c71c71cp-4;
  p = p * s2 + 0x1.2492492492492p-3;
  p = p * s2 + 0x1.999999999999ap-3;
  p = p * s2 + 0x1.5555555555555p-2;
  p = p * s2 + 0x1.0000000000000p+0;
  const double t = s * p;
  return (double)e * 0x1.62e42fefa39efp-1 + 2.0 * t;
}

// cos(2 pi t) for t in [0, 1]: exact reductions to [0, 1/8] of a turn, then the cosine or sine
// series (10 terms) on |x| <= pi/4.
THC_HD inline double gen_cos_turns(double t) {
  THC_NOCONTRACT
  double a = t >= 0.5 ? 1.0 - t : t;
  const bool neg = a > 0.25;
  if (neg) a = 0.5 - a;
  const bool use_sin = a > 0.125;
  if (use_sin) a = 0.25 - a;
  const double x = a * 0x1.921fb54442d18p+2;
  const double x2 = x * x;
  double c = -0x1.6827863b97d97p-53;
  c = c * x2 + 0x1.ae7f3e733b81fp-45;
  c = c * x2 + -0x1.93974a8c07c9dp-37;
  c = c * x2 + 0x1.1eed8eff8d898p-29;
  c = c * x2 + -0x1.27e4fb7789f5cp-22;
  c = c * x2 + 0x1.a01a01a01a01ap-16;
  c = c * x2 + -0x1.6c16c16c16c17p-10;
  c = c * x2 + 0x1.5555555555555p-5;
  c = c * x2 + -0x1.0000000000000p-1;
  c = c * x2 + 0x1.0000000000000p+0;
  double s = -0x1.2f49b46814157p-57;
  s = s * x2 + 0x1.952c77030ad4ap-49;
  s = s * x2 + -0x1.ae7f3e733b81fp-41;
  s = s * x2 + 0x1.6124613a86d09p-33;
  s = s * x2 + -0x1.ae64567f544e4p-26;
  s = s * x2 + 0x1.71de3a556c734p-19;
  s = s * x2 + -0x1.a01a01a01a01ap-13;
  s = s * x2 + 0x1.1111111111111p-7;
  s = s * x2 + -0x1.5555555555555p-3;
  s = s * x2 + 0x1.0000000000000p+0;
  const double sn = x * s;
  const double r = use_sin ? sn : c;
  return neg ? -r : r;
}

// e^x for x in about [-700, 0]: x = n ln 2 + r, n = floor(x / ln 2 + 1/2) (ln 2 in two parts),
// 15 terms of the series of e^r, scaled by 2^n exactly.
THC_HD inline double gen_exp(double x) {
  THC_NOCONTRACT
  const double n = __builtin_floor(x * 0x1.71547652b82fep+0 + 0.5);
  const double r = (x - n * 0x1.62e42fee00000p-1) - n * 0x1.a39ef00000000p-33;
  double p = 0x1.93974a8c07c9dp-37;
  p = p * r + 0x1.6124613a86d09p-33;
  p = p * r + 0x1.1eed8eff8d898p-29;
  p = p * r + 0x1.ae64567f544e4p-26;
  p = p * r + 0x1.27e4fb7789f5cp-22;
  p = p * r + 0x1.71de3a556c734p-19;
  p = p * r + 0x1.a01a01a01a01ap-16;
  p = p * r + 0x1.a01a01a01a01ap-13;
  p = p * r + 0x1.6c16c16c16c17p-10;
  p = p * r + 0x1.1111111111111p-7;
  p = p * r + 0x1.5555555555555p-5;
  p = p * r + 0x1.5555555555555p-3;
  p = p * r + 0x1.0000000000000p-1;
  p = p * r + 0x1.0000000000000p+0;
  p = p * r + 0x1.0000000000000p+0;
  return p * from_bits((uint64_t)(1023 + (int64_t)n) << 52);
}

// Standard normal number idx of the stream with key k (Box-Muller of uniforms 2 idx, 2 idx + 1).
THC_HD inline double normal(uint64_t k, uint64_t idx) {
  THC_NOCONTRACT
  const double u1 = uniform(k, 2 * idx), u2 = uniform(k, 2 * idx + 1);
  return __builtin_sqrt(-2.0 * gen_log(u1)) * gen_cos_turns(u2);
}

// e^(-K/decay): the decay of Cholesky vector K.
THC_HD inline double decay_factor(int64_t K, double decay) {
  THC_NOCONTRACT
  return gen_exp(-(double)K / decay);
}

}  // namespace thc_synth
