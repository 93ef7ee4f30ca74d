// fastpow.h -- ln x and x^y for x > 0 in FP64, composed of the series of
// atanh (for the logarithm) and of exp (for 2^t), each truncated where its
// next term falls below 2^-60 of the sum.
//   * pow_pos: the FP64 edge probability of Eq. (1) raises its ratio to the
//     power 1/T once per tested pair (type-I tests, type-II candidates).  This
//     takes about a quarter of the instructions of the math library's pow.
//     Its relative error stays below 2^-52 (6 + 2 |y log2 x|); for p <= 1
//     that is an absolute error below 1e-15, so a decision U < p taken with it
//     can differ from the exact one only for |U - p| < 1e-15.
//   * log_pos: the logarithm of a type-II draw's uniform, once per geometric
//     skip (Sec. 3.2), with a relative error below 2^-52 * 3.  A skip length
//     floor(ln S / ln(1 - pbar)) can then differ from the exact one only where
//     the quotient lies within about 1e-15 (relative) of an integer.
// The host test checks both against the C library's pow and log.  No IEEE
// special cases beyond x <= 0 and x = inf are handled: callers pass positive
// finite arguments (and cap probabilities at 1).
//
// Every step is an explicit fma, a correctly rounded operation or an exact
// one (frexp, ldexp, rint, z - rint z), and the library is built with
// -ffp-contract=off, so host and device builds give the same bits.
#pragma once

#include <hip/hip_runtime.h>
#include <math.h>

namespace hg {

// x = m 2^k with m in [sqrt(1/2), sqrt(2)) (x > 0 finite); returns k and
// s P with ln m = 2 s P: s = (m - 1) / (m + 1), |s| < 0.1716, and
// P = atanh(s) / s = sum_j s^2j / (2j + 1), j <= 10 (the next term is below
// 0.0295^11 / 23)
__host__ __device__ inline double atanh_part(double x, int* kk) {
  int k = 0;
  double m = frexp(x, &k);
  if (m < 0.70710678118654752440) {
    m = 2.0 * m;
    k -= 1;
  }
  *kk = k;
  const double f = m - 1.0;
  const double s = f / (m + 1.0);
  const double s2 = s * s;
  double P = 1.0 / 21.0;
  P = fma(P, s2, 1.0 / 19.0);
  P = fma(P, s2, 1.0 / 17.0);
  P = fma(P, s2, 1.0 / 15.0);
  P = fma(P, s2, 1.0 / 13.0);
  P = fma(P, s2, 1.0 / 11.0);
  P = fma(P, s2, 1.0 / 9.0);
  P = fma(P, s2, 1.0 / 7.0);
  P = fma(P, s2, 1.0 / 5.0);
  P = fma(P, s2, 1.0 / 3.0);
  P = fma(P, s2, 1.0);
  return s * P;
}

// ln x = k ln 2 + 2 s P, with ln 2 split into a head of 32 significant bits
// (k ln2_hi is exact for |k| < 2^21) and the rest
__host__ __device__ inline double log_pos(double x) {
  if (!(x < INFINITY)) return INFINITY;
  if (!(x > 0.0)) return -INFINITY;
  int k = 0;
  const double sp = atanh_part(x, &k);
  const double ln2_hi = 0x1.62e42fee00000p-1;
  const double ln2_lo = 1.9082149292705877e-10;  // ln 2 - ln2_hi, rounded
  return fma((double)k, ln2_hi, fma((double)k, ln2_lo, 2.0 * sp));
}

__host__ __device__ inline double pow_pos(double x, double y) {
  if (!(x < INFINITY)) return INFINITY;
  if (!(x > 0.0)) return 0.0;
  // log2 x = k + (2 / ln 2) s P
  int k = 0;
  const double sp = atanh_part(x, &k);
  const double lg = fma(sp, 2.0 * 1.44269504088896340736, (double)k);
  const double z = y * lg;
  if (z < -1100.0) return 0.0;
  if (z > 1100.0) return INFINITY;
  // 2^z = 2^n e^r, n = rint z, r = (z - n) ln 2 in [-0.35, 0.35]:
  // e^r = sum_k r^k / k!, k <= 13 (the next term is below 0.35^14 / 14!)
  const double n = rint(z);
  const double r = (z - n) * 0.69314718055994530942;
  double e = 1.0 / 6227020800.0;
  e = fma(e, r, 1.0 / 479001600.0);
  e = fma(e, r, 1.0 / 39916800.0);
  e = fma(e, r, 1.0 / 3628800.0);
  e = fma(e, r, 1.0 / 362880.0);
  e = fma(e, r, 1.0 / 40320.0);
  e = fma(e, r, 1.0 / 5040.0);
  e = fma(e, r, 1.0 / 720.0);
  e = fma(e, r, 1.0 / 120.0);
  e = fma(e, r, 1.0 / 24.0);
  e = fma(e, r, 1.0 / 6.0);
  e = fma(e, r, 0.5);
  e = fma(e, r, 1.0);
  e = fma(e, r, 1.0);
  return ldexp(e, (int)n);
}

}  // namespace hg
