// Double-precision logarithms for the solver kernels.
//
// The sweep evaluates log2(1 + x) once per (RRH, subcarrier, user) triple
// and once or twice more per selected user; the general-purpose library
// versions carry extra-precision arithmetic that makes them several times
// longer than needed here.  These are table-driven, after P. T. P. Tang,
// "Table-driven implementation of the logarithm function in IEEE
// floating-point arithmetic", ACM TOMS 16(4), 1990:
//
//   x = 2^e m,  sqrt(1/2) <= m < sqrt(2),   c = j/128 the nearest multiple,
//   log x = e ln 2 - log(1/c) + log(1 + r),  r = m (1/c) - 1,  |r| < 0.0056,
//
// where 1/c is the double in the table (logtab.h) and -log(1/c) of that very
// double is tabulated as a head and a tail, so r = fma(m, 1/c, -1) carries a
// single rounding; log(1 + r) is its series through r^8 (truncation below
// 2^-70 of the result).  ln 2 is split into a 32-bit head (e ln2_hi exact)
// and a tail, and the heads are added in one rounding: within about 1 ulp,
// and exact where c = 1 and e = 0 (x near 1).  log1p(x) adds to log(1 + x)
// the first-order correction for the rounding of 1 + x,
// (x - ((1 + x) - 1)) / (1 + x), which keeps small arguments accurate.
#pragma once

#include <hip/hip_runtime.h>
#include <math.h>

#include "logtab.h"

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
  m = low ? 2.0 * m : m;  // [sqrt(1/2), sqrt(2))
  e = low ? e - 1 : e;
  // nearest c = j/128 (91 <= j <= 181; the clamp only matters for 0, inf, NaN)
  const int j = min(max((int)(m * 128.0 + 0.5), kLogTabJ0), kLogTabJ0 + 90);
  const double* tb = kLogTab[j - kLogTabJ0];
  const double r = fma(m, tb[0], -1.0);
  double p = -1.0 / 8.0;
  p = fma(p, r, 1.0 / 7.0);
  p = fma(p, r, -1.0 / 6.0);
  p = fma(p, r, 1.0 / 5.0);
  p = fma(p, r, -1.0 / 4.0);
  p = fma(p, r, 1.0 / 3.0);
  p = fma(p, r, -0.5);
  const double lr = fma(r * r, p, r);  // log(1 + r)
  const double fe = (double)e;
  const double hi = fma(fe, kLn2Hi, tb[1]);
  const double lo = fma(fe, kLn2Lo, tb[2]) + lr;
  const double res = hi + lo;
  if (x == 0.0) return -INFINITY;
  return x < INFINITY ? res : x;
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
