// crmath.hpp -- exp, log and pow in FP64 for the kernels, rounded from a
// double-double evaluation.
//
// The integrators' control decisions (accept/reject, stage counts) depend on
// round-off: a one-ulp change in a step size can flip a later decision.  The
// kernels therefore evaluate every transcendental function to the exact value
// rounded to the nearest double wherever a double-double evaluation can
// decide that rounding, which makes their results a function of the inputs
// alone rather than of a particular math library.
//
// Method: table-driven argument reduction (Tang, ACM TOMS 15 (1989) for exp,
// 16 (1990) for log) carried out in double-double arithmetic built on the
// error-free transformations TwoSum (Knuth) and TwoProd via FMA (Dekker).
// The double-double result has relative error below about 2^-88; its final
// rounding is the correctly rounded value unless the exact value lies that
// close to a rounding midpoint, about 2^-35 of calls (no such input is known,
// and there is no slower fallback that would decide them: these functions are
// not proven correctly rounded).  exp results in the subnormal range are scaled after rounding (a
// possible double rounding there).  Functions are __host__ __device__ so that
// the identical code can be checked on the CPU.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <string.h>

#include "crmath_tables.hpp"

#define RKMI_HD __host__ __device__ __forceinline__

namespace rkmi {
namespace crm {

struct dd {
  double hi, lo;
};

RKMI_HD bool is_nan(double x) { return x != x; }
RKMI_HD bool is_finite(double x) { return fabs(x) <= 0x1.fffffffffffffp+1023; }

RKMI_HD uint64_t bits_of(double x) {
  uint64_t u;
  memcpy(&u, &x, sizeof u);
  return u;
}

RKMI_HD double from_bits(uint64_t u) {
  double x;
  memcpy(&x, &u, sizeof x);
  return x;
}

// s + e = a + b exactly
RKMI_HD dd two_sum(double a, double b) {
  const double s = a + b;
  const double bb = s - a;
  const double e = (a - (s - bb)) + (b - bb);
  return {s, e};
}

// s + e = a + b exactly, provided |a| >= |b| or a == 0
RKMI_HD dd fast_two_sum(double a, double b) {
  const double s = a + b;
  return {s, b - (s - a)};
}

// p + e = a * b exactly
RKMI_HD dd two_prod(double a, double b) {
  const double p = a * b;
  return {p, fma(a, b, -p)};
}

RKMI_HD dd dd_mul(dd a, dd b) {
  const dd p = two_prod(a.hi, b.hi);
  const double e = p.lo + (a.hi * b.lo + a.lo * b.hi);
  return fast_two_sum(p.hi, e);
}

// 2^m for m in [-1022, 1023]
RKMI_HD double pow2i(int m) { return from_bits((uint64_t)(m + 1023) << 52); }

RKMI_HD double scale2(double x, int m) {
  if (m > 1023) {
    x *= pow2i(1023);
    m -= 1023;
    if (m > 1023) m = 1023;
  } else if (m < -1022) {
    x *= pow2i(-1022);
    m += 1022;
    if (m < -1022) m = -1022;
  }
  return x * pow2i(m);
}

// exp(zh + zl) = 2^m (R.hi + R.lo) as a double-double R in [1 - 2^-11, 2 + 2^-10]
// and an exponent m, for zh within exp_dd's finite range and |zl| <= ulp(zh).
RKMI_HD dd exp_core(double zh, double zl, int& m_out) {
  // z = k ln2/1024 + r, |r| <= ln2/2048
  const double kd = rint(zh * kInvL);
  const double rh = zh - kd * kL1;                 // exact
  const dd p = two_prod(kd, kL2);
  const dd s = two_sum(rh, -p.hi);
  const double lo = ((s.lo - p.lo) - kd * kL3) + zl;
  const dd r = two_sum(s.hi, lo);
  // exp(r) = 1 + r + r^2/2 + r^3/6 + ... + r^7/5040
  const double x = r.hi;
  dd q = two_prod(x, x);
  q.lo += 2.0 * x * r.lo;
  const double tail =
      x * q.hi *
      (0x1.5555555555555p-3 +
       x * (0x1.5555555555555p-5 +
            x * (0x1.1111111111111p-7 + x * (0x1.6c16c16c16c17p-10 + x * 0x1.a01a01a01a01ap-13))));
  const dd e1 = fast_two_sum(1.0, x);
  const dd e2 = two_sum(e1.hi, 0.5 * q.hi);
  const double elo = e1.lo + e2.lo + (r.lo + (0.5 * q.lo + tail));
  const dd E = fast_two_sum(e2.hi, elo);
  // 2^(k/1024) = 2^m 2^(j1/32) 2^(j2/1024)
  const int64_t k = (int64_t)kd;
  const int64_t m = k >> 10;
  const int jj = (int)(k - (m << 10));
  const int j1 = jj >> 5, j2 = jj & 31;
  const dd T = dd_mul(dd{kExpT1[2 * j1], kExpT1[2 * j1 + 1]}, dd{kExpT2[2 * j2], kExpT2[2 * j2 + 1]});
  m_out = (int)m;
  return dd_mul(T, E);
}

constexpr double kExpMaxArg = 709.782712893384;
constexpr double kExpMinArg = -745.1332191019412;

// exp(zh + zl) rounded to nearest, |zl| <= ulp(zh).
RKMI_HD double exp_dd(double zh, double zl) {
  if (zh != zh) return zh;
  if (zh > kExpMaxArg) return __builtin_huge_val();
  if (zh < kExpMinArg) return 0.0;
  int m = 0;
  const dd R = exp_core(zh, zl, m);
  return scale2(R.hi + R.lo, m);
}

// log1p(u) for a double-double u with |u| <= 2^-9:
// u - u^2/2 + u^3/3 (double-double) - u^4/4 + ... + u^11/11 (double).
RKMI_HD dd log1p_small(double uh, double ul) {
  dd a = two_prod(uh, uh);
  a.lo += 2.0 * uh * ul;
  dd b = two_prod(a.hi, uh);
  b.lo += a.lo * uh + a.hi * ul;
  const double b3 = b.hi / 3.0;
  const double b3l = (fma(-3.0, b3, b.hi) + b.lo) / 3.0;
  const double tail =
      a.hi * a.hi *
      (-0.25 +
       uh * (0.2 +
             uh * (-0x1.5555555555555p-3 +
                   uh * (0x1.2492492492492p-3 +
                         uh * (-0.125 + uh * (0x1.c71c71c71c71cp-4 +
                                              uh * (-0.1 + uh * 0x1.745d1745d1746p-4)))))));
  const dd s1 = two_sum(uh, -0.5 * a.hi);
  const dd s2 = two_sum(s1.hi, b3);
  const double slo = s1.lo + s2.lo + ((ul - 0.5 * a.lo) + (b3l + tail));
  return two_sum(s2.hi, slo);
}

// log(x) as a double-double, x > 0 finite: absolute error below about 2^-95,
// and relative error below about 2^-80 where |x - 1| < 2^-9.
RKMI_HD dd log_dd(double x) {
  if (fabs(x - 1.0) < 0x1p-9) return log1p_small(x - 1.0, 0.0);  // x - 1 is exact here
  int e = 0;
  uint64_t u = bits_of(x);
  int ex = (int)((u >> 52) & 0x7ff);
  if (ex == 0) {  // subnormal: scale into the normal range
    x *= 0x1p54;
    u = bits_of(x);
    ex = (int)((u >> 52) & 0x7ff);
    e = -54;
  }
  e += ex - 1023;
  const double mnt = from_bits((u & 0x000fffffffffffffULL) | 0x3ff0000000000000ULL);  // [1, 2)
  const int j = (int)((u >> 44) & 0xff);
  // u = mnt * inv_j - 1 exactly as a double-double, |u| <= 2^-9
  const dd pr = two_prod(mnt, kLogInv[j]);
  const dd uu = two_sum(pr.hi - 1.0, pr.lo);
  const dd S = log1p_small(uu.hi, uu.lo);
  // e ln2 + (-log inv_j) + log1p(u)
  const double ed = (double)e;
  const double eh = ed * kLn2a;  // exact
  const dd el = two_prod(ed, kLn2b);
  const dd t1 = two_sum(eh, kLogT[2 * j]);
  const dd t2 = two_sum(t1.hi, el.hi);
  const dd t3 = two_sum(t2.hi, S.hi);
  const double lo = ((t1.lo + t2.lo) + t3.lo) + ((kLogT[2 * j + 1] + (el.lo + ed * kLn2c)) + S.lo);
  return two_sum(t3.hi, lo);
}

// exp(x), rounded as the header describes.  A first evaluation: the reduction of exp_dd
// (r + rl = x - k ln2/1024 to 2^-115), 1 + r + (rl (1 + r) + r^2 (1/2 + r/6 +
// r^2/24 + r^3/120)) as a double-double (relative error below 2^-74.5: the
// truncation r^6/720 < 2^-78.5 and the rounding of the r^2 terms), times the
// double-double 2^(j/1024): relative error below 2^-74 in all.  When the
// double-double result R lies farther than 2^-70 from the midpoints around
// R.hi, the exact value rounds to R.hi; that fails for about 2^-17 of inputs
// (and where R.hi is a power of two), which take exp_dd, as do the ends of the
// range (subnormal results, overflow, NaN).
RKMI_HD double cr_exp(double x) {
  if (!(x > -708.3 && x < 709.7)) return exp_dd(x, 0.0);
  const double kd = rint(x * kInvL);
  const double rh = x - kd * kL1;                  // exact
  const dd p = two_prod(kd, kL2);
  const dd s = two_sum(rh, -p.hi);
  const double rl = (s.lo - p.lo) - kd * kL3;
  const double r = s.hi;
  const double q = (r * r) * (0.5 + r * (0x1.5555555555555p-3 +
                                         r * (0x1.5555555555555p-5 + r * 0x1.1111111111111p-7)));
  const dd e1 = fast_two_sum(1.0, r);
  const dd E = fast_two_sum(e1.hi, e1.lo + ((rl + rl * r) + q));
  const int64_t k = (int64_t)kd;
  const int64_t m = k >> 10;
  const int jj = (int)(k - (m << 10));
  const int j1 = jj >> 5, j2 = jj & 31;
  const dd T = dd_mul(dd{kExpT1[2 * j1], kExpT1[2 * j1 + 1]}, dd{kExpT2[2 * j2], kExpT2[2 * j2 + 1]});
  const dd R = dd_mul(T, E);
  const double half_ulp = R.hi >= 2.0 ? 0x1p-52 : (R.hi >= 1.0 ? 0x1p-53 : 0x1p-54);
  if (fabs(R.lo) < half_ulp - 0x1p-70 && R.hi != 1.0 && R.hi != 2.0) return scale2(R.hi, (int)m);
  return exp_dd(x, 0.0);
}

RKMI_HD double cr_log(double x) {
  if (x != x) return x;
  if (x < 0.0) return __builtin_nan("");
  if (x == 0.0) return -__builtin_huge_val();
  if (x == __builtin_huge_val()) return x;
  const dd L = log_dd(x);
  return L.hi + L.lo;
}

// x^y for x > 0 finite from a precomputed log_dd(x).
RKMI_HD double pow_from_log(dd L, double y) {
  dd z = two_prod(y, L.hi);
  z.lo += y * L.lo;
  return exp_dd(z.hi, z.lo);
}

// x^y with the special values of C99 Annex F (y finite and not an integer
// in the cases the integrators produce).
RKMI_HD double cr_pow(double x, double y) {
  if (y == 0.0) return 1.0;
  if (x == 1.0) return 1.0;
  if (x != x || y != y) return x + y;
  const double inf = __builtin_huge_val();
  const bool y_int = (rint(y) == y);
  const bool y_odd = y_int && (fabs(y) < 0x1p53) && (fmod(y, 2.0) != 0.0);
  if (x == 0.0) {
    if (y < 0.0) return (y_odd && bits_of(x) >> 63) ? -inf : inf;
    return (y_odd && bits_of(x) >> 63) ? -0.0 : 0.0;
  }
  if (y == inf || y == -inf) {
    const double ax = fabs(x);
    if (ax == 1.0) return 1.0;
    return ((ax > 1.0) == (y > 0.0)) ? inf : 0.0;
  }
  if (x == inf) return y > 0.0 ? inf : 0.0;
  if (x == -inf) {
    if (y > 0.0) return y_odd ? -inf : inf;
    return y_odd ? -0.0 : 0.0;
  }
  if (x < 0.0) {
    if (!y_int) return __builtin_nan("");
    const double r = pow_from_log(log_dd(-x), y);
    return y_odd ? -r : r;
  }
  return pow_from_log(log_dd(x), y);
}

// x^y for y = RN(1/3) and, when kSquare, x^(2y) (2y = RN(2/3)), for finite
// x >= 0.  Since y = 1/3 - 2^-54/3 exactly,
//   x^y = cbrt(x) x^(-2^-54/3) = cbrt(x) (1 + u + u^2/2 + ...),
//   u = -(2^-54/3) ln x,  |u| < 1.4e-14,
// and x^(2y) is the square of x^y.  x = t 2^(3q) with t in [1, 8): t^(-1/3)
// from a degree-4 fit of m^(-1/3) on [1, 2) (relative error 8.8e-5; the fit
// is ours) and two Newton steps z <- z + z (1 - t z^3) / 3, then cbrt(t) =
// t z^2 and one Newton step for the cube root in double-double arithmetic (the
// residual c^3 - t formed exactly with TwoProd).  ln x = e ln2 + 2 atanh(s),
// s = (m - 1)/(m + 1), needs absolute accuracy of only about 1e-11 here (the
// series to s^13 gives 4e-13).  The double-double result has relative error
// below about 2^-90, so both roundings give the correctly rounded values except
// for about 2^-37 of calls (the exact value that close to a midpoint).
constexpr double kThird = 0x1.5555555555555p-2;            // RN(1/3)
constexpr double kThirdDefect = 0x1.5555555555555p-56;     // 1/3 - RN(1/3), rounded
constexpr double kCbrtFit[5] = {0x1.bf460be1acba9p-1, -0x1.8d16b63ef59afp-3,
                                0x1.60afbeaf93db8p-4, -0x1.9213bd85642a6p-5,
                                0x1.c40554f37ed1bp-6};     // m^(-1/3) in powers of m - 3/2
constexpr double kCbrtHalf = 0x1.965fea53d6e3dp-1;         // RN(2^(-1/3))
constexpr double kCbrtQuarter = 0x1.428a2f98d728bp-1;      // RN(2^(-2/3))
constexpr double kSqrt2 = 0x1.6a09e667f3bcdp+0;
constexpr double kLn2d = 0x1.62e42fefa39efp-1;

// ln(m 2^e) for m in [1, 2) to an absolute error of about 4e-13: e ln2 +
// 2 atanh(s), s = (m' - 1)/(m' + 1) with m' = m or m / 2 in [sqrt(1/2),
// sqrt(2)), the series to s^13.  Enough for the small correction factors
// x^(1/3 - RN(1/3)) and x^(RN(0.2) - 1/5) below.
RKMI_HD double log_rough(double m, int e) {
  double mm = m;
  int ee = e;
  if (mm > kSqrt2) {
    mm = 0.5 * mm;
    ee += 1;
  }
  const double sv = (mm - 1.0) / (mm + 1.0);
  const double s2 = sv * sv;
  const double lnm =
      2.0 * sv *
      (1.0 + s2 * (0x1.5555555555555p-2 +
                   s2 * (0.2 + s2 * (0x1.2492492492492p-3 +
                                     s2 * (0x1.c71c71c71c71cp-4 +
                                           s2 * (0x1.745d1745d1746p-4 + s2 * 0x1.3b13b13b13b14p-4))))));
  return (double)ee * kLn2d + lnm;
}

// x = m 2^e with m in [1, 2), for finite x > 0 (subnormals scaled).
RKMI_HD void split_normal(double x, double& m, int& e) {
  uint64_t b = bits_of(x);
  int ex = (int)(b >> 52);
  int sc = 0;
  if (ex == 0) {
    b = bits_of(x * 0x1p54);
    ex = (int)(b >> 52);
    sc = -54;
  }
  e = ex - 1023 + sc;
  m = from_bits((b & 0x000fffffffffffffULL) | 0x3ff0000000000000ULL);
}

template <bool kSquare>
RKMI_HD void pow_third(double x, double& p1, double& p2) {
  if (x == 0.0 || x == 1.0) {
    p1 = p2 = x;
    return;
  }
  if (!(x > 0.0) || !is_finite(x)) {
    p1 = cr_pow(x, kThird);
    p2 = kSquare ? cr_pow(x, 2.0 * kThird) : 0.0;
    return;
  }
  double m;
  int e;
  split_normal(x, m, e);          // x = m 2^e, m in [1, 2)
  int q = e / 3, r = e - 3 * q;
  if (r < 0) {
    r += 3;
    q -= 1;
  }
  const double t = r == 0 ? m : (r == 1 ? 2.0 * m : 4.0 * m);
  const double d = m - 1.5;
  double z = kCbrtFit[0] + d * (kCbrtFit[1] + d * (kCbrtFit[2] + d * (kCbrtFit[3] + d * kCbrtFit[4])));
  z = z * (r == 0 ? 1.0 : (r == 1 ? kCbrtHalf : kCbrtQuarter));
  z = z + z * (1.0 - t * (z * z * z)) * kThird;
  z = z + z * (1.0 - t * (z * z * z)) * kThird;
  const double c = t * (z * z);
  const dd c2 = two_prod(c, c);
  const dd c3 = two_prod(c, c2.hi);
  const double res = (c3.hi - t) + (c3.lo + c * c2.lo);
  const double delta = res * (z * z) * kThird;   // (c^3 - t) / (3 c^2)
  const double u = -kThirdDefect * log_rough(m, e);
  const dd P = fast_two_sum(c, c * (u + 0.5 * u * u) - delta);
  p1 = scale2(P.hi + P.lo, q);
  if (kSquare) {
    const dd P2 = dd_mul(P, P);
    p2 = scale2(P2.hi + P2.lo, 2 * q);
  } else {
    p2 = 0.0;
  }
}

// x^RN(1/3) and x^RN(2/3) for finite x >= 0 (rounded as cr_pow).
RKMI_HD void pow_third_pair(double x, double& p1, double& p2) { pow_third<true>(x, p1, p2); }

// x^RN(1/3) for finite x >= 0 (rounded as cr_pow).
RKMI_HD double pow_third_one(double x) {
  double p1, p2;
  pow_third<false>(x, p1, p2);
  return p1;
}

// (1 + d)^-y for |d| < 2^-40 and 0 < y < 1: 1 - y d + (y (y + 1) / 2) d^2
// (the next term is below 2^-120) in double-double, rounded once.  Near 1 the
// exact powers can lie within about 2^-104 of a rounding midpoint (x = 1 +
// k 2^-52 gives 1 - k 2^-54 + O(k^2 2^-104) for y = 1/4), closer than the
// root-and-Newton evaluations below resolve.
RKMI_HD double pow_near_one(double d, double y) {
  const dd p = two_prod(y, d);
  const dd r = fast_two_sum(1.0, -p.hi);
  const double c2 = 0.5 * (y * (y + 1.0));
  return r.hi + ((r.lo - p.lo) + c2 * (d * d));
}

// x^-0.25 for finite x > 0, rounded as cr_pow(x, -0.25): x =
// t 2^(4q) with t in [1, 16); a0 = 1 / sqrt(sqrt(t)) (relative error below
// 2^-50), then one Newton step for t a^4 = 1 in double-double, a = a0 - a0
// (t a0^4 - 1) / 4 with the residual formed exactly by TwoProd: relative
// error below about 2^-98 before the final rounding.
RKMI_HD double pow_minus_quarter(double x) {
  if (!(x > 0.0) || !is_finite(x)) return cr_pow(x, -0.25);
  double m;
  int e;
  split_normal(x, m, e);
  const int q = e >> 2;                       // floor(e / 4)
  const double t = m * (double)(1 << (e - 4 * q));
  // near a power of 16 (t near 1 or 16) the series
  if (t - 1.0 < 0x1p-40) return scale2(pow_near_one(t - 1.0, 0.25), -q);
  if (16.0 - t < 0x1p-36) return scale2(pow_near_one(0.0625 * t - 1.0, 0.25), -q - 1);
  const double a0 = 1.0 / sqrt(sqrt(t));
  const dd a2 = two_prod(a0, a0);
  const dd a4 = two_prod(a2.hi, a2.hi);
  const double a4lo = a4.lo + 2.0 * a2.hi * a2.lo;
  const dd p = two_prod(t, a4.hi);
  const double res = (p.hi - 1.0) + (p.lo + t * a4lo);
  const dd A = fast_two_sum(a0, -0.25 * (a0 * res));
  return scale2(A.hi + A.lo, -q);
}

// x^-RN(0.2) for finite x > 0, rounded as cr_pow(x, -0.2).  Since
// RN(0.2) = 1/5 + 2^-54/5 exactly, x^-RN(0.2) = x^(-1/5) (1 - u + u^2/2 ...)
// with u = (2^-54/5) ln x, |u| < 8.3e-15.  x = t 2^(5q) with t in [1, 32):
// t^(-1/5) from a degree-4 fit of m^(-1/5) on [1, 2) (relative error 4.2e-5;
// the fit is ours) times 2^(-r/5), two Newton steps z <- z + z (1 - t z^5)/5
// and one in double-double; relative error below about 2^-95.
constexpr double kFifthDefect = 0x1.999999999999ap-57;       // RN(0.2) - 1/5, rounded
constexpr double kFifthFit[5] = {0x1.d81ea442f789fp-1, -0x1.f71b3cd67e5e7p-4,
                                 0x1.9206823b82378p-5, -0x1.ad6fd51751e20p-6,
                                 0x1.d2a8f56f71fa3p-7};       // m^(-1/5) in powers of m - 3/2
constexpr double kFifthRoot2[5] = {0x1.0000000000000p+0, 0x1.bdb8cdadbe120p-1,
                                   0x1.8406003b2ae5cp-1, 0x1.51cb453b9536cp-1,
                                   0x1.2611186bae674p-1};     // RN(2^(-r/5))

RKMI_HD double pow_minus_fifth(double x) {
  if (!(x > 0.0) || !is_finite(x)) return cr_pow(x, -0.2);
  // near 1 the series (near other powers of 32 the factor x^-(RN(0.2) - 1/5)
  // moves the value off the midpoints)
  if (fabs(x - 1.0) < 0x1p-40) return pow_near_one(x - 1.0, 0.2);
  double m;
  int e;
  split_normal(x, m, e);
  int q = e / 5, r = e - 5 * q;
  if (r < 0) {
    r += 5;
    q -= 1;
  }
  const double t = m * (double)(1 << r);
  const double d = m - 1.5;
  double z = kFifthFit[0] + d * (kFifthFit[1] + d * (kFifthFit[2] + d * (kFifthFit[3] + d * kFifthFit[4])));
  z = z * kFifthRoot2[r];
  for (int it = 0; it < 2; ++it) {
    const double z2 = z * z;
    z = z + z * (1.0 - t * (z2 * z2 * z)) * 0.2;
  }
  const dd z2 = two_prod(z, z);
  const dd z4 = two_prod(z2.hi, z2.hi);
  const double z4lo = z4.lo + 2.0 * z2.hi * z2.lo;
  const dd z5 = two_prod(z4.hi, z);
  const double z5lo = z5.lo + z4lo * z;
  const dd p = two_prod(t, z5.hi);
  const double res = (p.hi - 1.0) + (p.lo + t * z5lo);
  const double u = kFifthDefect * log_rough(m, e);
  const dd P = fast_two_sum(z, z * (0.5 * u * u - u) - 0.2 * (z * res));
  return scale2(P.hi + P.lo, -q);
}

}  // namespace crm
}  // namespace rkmi
