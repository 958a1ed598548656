// FP64 natural logarithm and exponential for the FP64 sampling path: about a
// third and a half of the instructions of the device library's versions, at an
// error of a few units in the last place (the device library's log evaluates in
// double-double arithmetic, which the lamination's 1e-12 energy bar does not
// need).  Both are written from the textbook reductions, every product-sum as an
// explicit fma and every quotient as an IEEE division, so that a host build of
// this header (the CPU accuracy test) computes the same bits as the device:
//
//   log x:  x = m 2^e with m in [sqrt(1/2), sqrt(2)), f = m - 1 (exact),
//           s = f / (2 + f), z = s^2; log m = log((1 + s)/(1 - s)) = 2 atanh s =
//           2s + s R(z) with R(z) = sum_{k>=1} 2 z^k / (2k + 1), rewritten with
//           2s = f - s f as f - s (f - R(z)); |s| <= 0.1716, so nine terms of
//           R leave a truncation below 2^-55 relative.  log x = e ln2 + log m
//           with ln 2 split in two so that e ln2_hi is exact.
//   exp v:  k = rint(v / ln2), r = v - k ln2 (two-part ln 2, |r| <= ln2 / 2),
//           e^r by its Taylor polynomial of degree 13 (truncation below 2^-57),
//           then 2^k by ldexp.
//
// Special values follow the C library: log of 0 is -inf, of a negative number
// or NaN is NaN, of +inf is +inf; exp of -inf (and below -746) is 0, of NaN is
// NaN.  exp is meant for arguments below 709 (the sampling path passes v <= 0).
#pragma once
#include <hip/hip_runtime.h>

#include <cmath>

namespace r1x {

// ln 2 = kLn2Hi + kLn2Lo: kLn2Hi is ln 2 truncated to 32 significant bits, so
// e kLn2Hi is exact for every exponent; kLn2Lo is the rounded remainder.
constexpr double kLn2Hi = 0x1.62e42feep-1;
constexpr double kLn2Lo = 0x1.a39ef35793c76p-33;
constexpr double kLog2e = 0x1.71547652b82fep+0;

__host__ __device__ inline double log_f64(double x) {
  int e;
  double m = std::frexp(x, &e);                       // x = m 2^e, m in [0.5, 1)
  const bool low = m < 0x1.6a09e667f3bcdp-1;          // sqrt(1/2)
  m = low ? m + m : m;
  e = low ? e - 1 : e;
  const double f = m - 1.0;
  const double s = f / (2.0 + f);
  const double z = s * s;
  // R(z) = sum_{k=1..9} 2 z^k / (2k + 1), coefficients 2/19 .. 2/3 (rounded to nearest)
  double R = 0x1.af286bca1af28p-4;
  R = std::fma(R, z, 0x1.e1e1e1e1e1e1ep-4);
  R = std::fma(R, z, 0x1.1111111111111p-3);
  R = std::fma(R, z, 0x1.3b13b13b13b14p-3);
  R = std::fma(R, z, 0x1.745d1745d1746p-3);
  R = std::fma(R, z, 0x1.c71c71c71c71cp-3);
  R = std::fma(R, z, 0x1.2492492492492p-2);
  R = std::fma(R, z, 0x1.999999999999ap-2);
  R = std::fma(R, z, 0x1.5555555555555p-1);
  R = R * z;
  const double lm = std::fma(-s, f - R, f);           // log m
  const double de = double(e);
  const double r = std::fma(de, kLn2Hi, std::fma(de, kLn2Lo, lm));
  const double inf = __builtin_huge_val();
  return (x > 0.0 && x < inf) ? r : (x == 0.0 ? -inf : (x == inf ? inf : __builtin_nan("")));
}

__host__ __device__ inline double exp_f64(double v) {
  const double w = v < -746.0 ? -746.0 : v;           // below: the result underflows to 0; NaN stays NaN
  const double k = std::rint(w * kLog2e);
  double r = std::fma(-k, kLn2Hi, w);
  r = std::fma(-k, kLn2Lo, r);
  // 1/j!, j = 13 .. 1 (rounded to nearest)
  double p = 0x1.6124613a86d09p-33;
  p = std::fma(p, r, 0x1.1eed8eff8d898p-29);
  p = std::fma(p, r, 0x1.ae64567f544e4p-26);
  p = std::fma(p, r, 0x1.27e4fb7789f5cp-22);
  p = std::fma(p, r, 0x1.71de3a556c734p-19);
  p = std::fma(p, r, 0x1.a01a01a01a01ap-16);
  p = std::fma(p, r, 0x1.a01a01a01a01ap-13);
  p = std::fma(p, r, 0x1.6c16c16c16c17p-10);
  p = std::fma(p, r, 0x1.1111111111111p-7);
  p = std::fma(p, r, 0x1.5555555555555p-5);
  p = std::fma(p, r, 0x1.5555555555555p-3);
  p = std::fma(p, r, 0.5);
  p = std::fma(p, r, 1.0);
  p = std::fma(p, r, 1.0);
  return std::ldexp(p, int(k));
}

}  // namespace r1x
