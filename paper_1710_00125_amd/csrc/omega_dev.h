// Device side of the Omega generator: i.i.d. N(0,1) entries (Section 3)
// from a counter-based generator, so that every entry is a pure function of
// (seed, index):
//   Philox4x64-10 (Salmon, Moraes, Dror, Shaw, SC'11), key (seed, stream 1),
//   counter (c, 0, 0, 0) -> 64-bit words w0..w3;
//   u1 = ((w0 >> 11) + 1) 2^-53 in (0,1], u2 = (w1 >> 11) 2^-53 in [0,1);
//   Box-Muller z0 = rho cos(2 pi u2), z1 = rho sin(2 pi u2),
//   rho = sqrt(-2 ln u1); (w2, w3) give z2, z3 the same way;
//   Omega(i, j) = z_{q mod 4} of counter q / 4, q = i n + j.
// ln, cos and sin are evaluated with a fixed sequence of correctly rounded
// IEEE double operations (no fused multiply-add), so the bits do not depend
// on a math library.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace rcp {
namespace omega_dev {

constexpr uint64_t kPhiloxM0 = 0xD2E7470EE14C6C93ull;
constexpr uint64_t kPhiloxM1 = 0xCA5A826395121157ull;
constexpr uint64_t kWeyl0 = 0x9E3779B97F4A7C15ull;
constexpr uint64_t kWeyl1 = 0xBB67AE8584CAA73Bull;
constexpr uint64_t kStreamOmega = 1;

__device__ __forceinline__ void philox4x64_10(uint64_t& x0, uint64_t& x1, uint64_t& x2,
                                              uint64_t& x3, uint64_t k0, uint64_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const uint64_t lo0 = kPhiloxM0 * x0, hi0 = __umul64hi(kPhiloxM0, x0);
    const uint64_t lo1 = kPhiloxM1 * x2, hi1 = __umul64hi(kPhiloxM1, x2);
    const uint64_t y0 = hi1 ^ x1 ^ k0;
    const uint64_t y2 = hi0 ^ x3 ^ k1;
    x0 = y0;
    x1 = lo1;
    x2 = y2;
    x3 = lo0;
    k0 += kWeyl0;
    k1 += kWeyl1;
  }
}

// ln 2 split in a 32-bit head (exact products with small integers) and tail
constexpr double kLn2Hi = 6.93147180369123816490e-01;
constexpr double kLn2Lo = 1.90821492927058770002e-10;
constexpr double kSqrtHalf = 0.70710678118654752440;
constexpr double kHalfPi = 1.57079632679489661923;

// ln x, x > 0: x = m 2^e, m in [sqrt(1/2), sqrt(2)); ln m = 2 atanh(s),
// s = (m-1)/(m+1), as 2 s (1 + s^2/3 + ... + s^20/21) by Horner.
__device__ inline double ln_fixed(double x) {
#pragma clang fp contract(off)
  int e;
  double m = frexp(x, &e);
  if (m < kSqrtHalf) {
    m = m * 2.0;
    e -= 1;
  }
  const double s = (m - 1.0) / (m + 1.0);
  const double z = s * s;
  double acc = 1.0 / 21.0;
  acc = acc * z + 1.0 / 19.0;
  acc = acc * z + 1.0 / 17.0;
  acc = acc * z + 1.0 / 15.0;
  acc = acc * z + 1.0 / 13.0;
  acc = acc * z + 1.0 / 11.0;
  acc = acc * z + 1.0 / 9.0;
  acc = acc * z + 1.0 / 7.0;
  acc = acc * z + 1.0 / 5.0;
  acc = acc * z + 1.0 / 3.0;
  acc = acc * z + 1.0;
  const double lnm = (2.0 * s) * acc;
  const double ed = (double)e;
  return ed * kLn2Hi + (lnm + ed * kLn2Lo);
}

// sin t, 0 <= t <= pi/4: Taylor series to t^19, Horner in t^2
__device__ inline double sin_poly(double t) {
#pragma clang fp contract(off)
  const double z = t * t;
  double acc = -1.0 / 121645100408832000.0;  // -1/19!
  acc = acc * z + 1.0 / 355687428096000.0;    // 1/17!
  acc = acc * z + -(1.0 / 1307674368000.0);   // -1/15!
  acc = acc * z + 1.0 / 6227020800.0;         // 1/13!
  acc = acc * z + -(1.0 / 39916800.0);        // -1/11!
  acc = acc * z + 1.0 / 362880.0;             // 1/9!
  acc = acc * z + -(1.0 / 5040.0);            // -1/7!
  acc = acc * z + 1.0 / 120.0;                // 1/5!
  acc = acc * z + -(1.0 / 6.0);               // -1/3!
  acc = acc * z + 1.0;
  return t * acc;
}

// cos t, 0 <= t <= pi/4: Taylor series to t^20, Horner in t^2
__device__ inline double cos_poly(double t) {
#pragma clang fp contract(off)
  const double z = t * t;
  double acc = 1.0 / 2432902008176640000.0;   // 1/20!
  acc = acc * z + -(1.0 / 6402373705728000.0);  // -1/18!
  acc = acc * z + 1.0 / 20922789888000.0;       // 1/16!
  acc = acc * z + -(1.0 / 87178291200.0);       // -1/14!
  acc = acc * z + 1.0 / 479001600.0;            // 1/12!
  acc = acc * z + -(1.0 / 3628800.0);           // -1/10!
  acc = acc * z + 1.0 / 40320.0;                // 1/8!
  acc = acc * z + -(1.0 / 720.0);               // -1/6!
  acc = acc * z + 1.0 / 24.0;                   // 1/4!
  acc = acc * z + -(1.0 / 2.0);                 // -1/2!
  acc = acc * z + 1.0;
  return acc;
}

// (cos 2 pi u, sin 2 pi u), u in [0,1): exact quadrant split, angle folded
// into [0, pi/4].
__device__ inline void cos_sin_2pi(double u, double& c, double& s) {
#pragma clang fp contract(off)
  const double f = u * 4.0;
  const double q = floor(f);
  const double g = f - q;
  const bool upper = g > 0.5;
  const double t = upper ? kHalfPi * (1.0 - g) : kHalfPi * g;
  const double st = sin_poly(t);
  const double ct = cos_poly(t);
  const double c1 = upper ? st : ct;
  const double s1 = upper ? ct : st;
  switch (((int)q) & 3) {
    case 0: c = c1; s = s1; break;
    case 1: c = -s1; s = c1; break;
    case 2: c = -c1; s = -s1; break;
    default: c = s1; s = -c1; break;
  }
}

__device__ inline void box_muller(uint64_t wa, uint64_t wb, double& z0, double& z1) {
#pragma clang fp contract(off)
  const double u1 = (double)((wa >> 11) + 1ull) * 0x1p-53;
  const double u2 = (double)(wb >> 11) * 0x1p-53;
  const double rho = sqrt(-2.0 * ln_fixed(u1));
  double c, s;
  cos_sin_2pi(u2, c, s);
  z0 = rho * c;
  z1 = rho * s;
}

// the four entries of counter c
// (stream kStreamOmega + j: the j-th fresh sketching matrix of Algorithm 2)
__device__ __forceinline__ void omega_quad(uint64_t seed, int64_t c, double z[4],
                                           uint64_t stream = kStreamOmega) {
  uint64_t x0 = (uint64_t)c, x1 = 0, x2 = 0, x3 = 0;
  philox4x64_10(x0, x1, x2, x3, seed, stream);
  box_muller(x0, x1, z[0], z[1]);
  box_muller(x2, x3, z[2], z[3]);
}

}  // namespace omega_dev
}  // namespace rcp
