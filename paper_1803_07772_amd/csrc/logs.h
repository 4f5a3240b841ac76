// Double-precision logarithms for the solver kernels.
//
// The sweep evaluates log2(1 + x) once per (RRH, subcarrier, user) triple
// and once or twice more per selected user; the general-purpose library
// versions carry extra-precision arithmetic that makes them several times
// longer than needed here.  These follow the classical reduction
//
//   x = 2^e m,  sqrt(1/2) <= m < sqrt(2),   log x = e ln 2 + log m,
//   log m = 2 atanh(s) = 2 (s + s^3/3 + s^5/5 + ...),  s = (m - 1)/(m + 1),
//
// with |s| < 0.1716, so the odd series through s^23 leaves a truncation
// below 2^-60 of the result.  m - 1 is exact, s carries about one rounding
// of (m + 1) and one of the quotient (a reciprocal estimate refined by a
// Newton step and a residual correction), and ln 2 is split into a 32-bit
// head (e ln2_hi exact) and a tail: the result is within about 2 ulp.
// log1p(x) adds to log(1 + x) the first-order correction for the rounding
// of 1 + x, (x - ((1 + x) - 1)) / (1 + x), which keeps small arguments
// accurate.
#pragma once

#include <hip/hip_runtime.h>
#include <math.h>

namespace alloc_logs {

constexpr double kLn2Hi = 0x1.62e42fee00000p-1;  // ln 2, leading 32 bits
constexpr double kLn2Lo = 0x1.a39ef35793c76p-33;  // ln 2 - kLn2Hi
constexpr double kSqrtHalf = 0x1.6a09e667f3bcdp-1;
constexpr double kInvLn2 = 0x1.71547652b82fep0;    // 1 / ln 2

// log x for x > 0; 0 gives -inf; +inf and NaN are returned unchanged.
__device__ __forceinline__ double log_d(double x) {
  int e;
  double m = frexp(x, &e);  // [1/2, 1)
  const bool low = m < kSqrtHalf;
  m = low ? 2.0 * m : m;
  e = low ? e - 1 : e;
  // s = (m - 1)/(m + 1) with the divisor in [1.7, 2.5): reciprocal estimate,
  // one Newton step, then the quotient's residual correction (no scaling
  // is needed in this range)
  const double a = m - 1.0, b = m + 1.0;
  double rb = __builtin_amdgcn_rcp(b);
  rb = fma(fma(-b, rb, 1.0), rb, rb);
  double s = a * rb;
  s = fma(fma(-b, s, a), rb, s);
  const double z = s * s;
  double p = 1.0 / 23.0;
  p = fma(p, z, 1.0 / 21.0);
  p = fma(p, z, 1.0 / 19.0);
  p = fma(p, z, 1.0 / 17.0);
  p = fma(p, z, 1.0 / 15.0);
  p = fma(p, z, 1.0 / 13.0);
  p = fma(p, z, 1.0 / 11.0);
  p = fma(p, z, 1.0 / 9.0);
  p = fma(p, z, 1.0 / 7.0);
  p = fma(p, z, 1.0 / 5.0);
  p = fma(p, z, 1.0 / 3.0);
  const double s2 = 2.0 * s;
  const double lm = fma(s2 * z, p, s2);  // 2s + 2s z p(z)
  const double fe = (double)e;
  const double r = fma(fe, kLn2Hi, fma(fe, kLn2Lo, lm));
  if (x == 0.0) return -INFINITY;
  return x < INFINITY ? r : x;
}

// log(1 + x) for x >= 0; +inf and NaN are returned unchanged.
__device__ __forceinline__ double log1p_d(double x) {
  const double u = 1.0 + x;
  const double c = (x - (u - 1.0)) * __builtin_amdgcn_rcp(u);  // a correction of relative size <= 2^-53
  const double r = log_d(u) + c;
  return x < INFINITY ? r : x;
}

__device__ __forceinline__ double log2_d(double x) { return log_d(x) * kInvLn2; }
__device__ __forceinline__ double log2_1p_d(double x) { return log1p_d(x) * kInvLn2; }

}  // namespace alloc_logs
