// Elementary functions of the step written for the GPU's issue budget.
//
// The header has no HIP dependency, so that a host compiler can build the
// same routine for its accuracy test.
#pragma once

#if defined(__HIPCC__)
#define CDI_HD __host__ __device__ __forceinline__
#else
#define CDI_HD inline
#endif

namespace cdi {

// Natural logarithm of a positive normal double, within 2 ulp.
//
// Argument reduction x = m 2^e with m in [1/sqrt 2, sqrt 2) (frexp and a
// doubling, both exact); log m = 2 atanh s with s = (m - 1)/(m + 1), so
// |s| <= 3 - 2 sqrt 2 < 0.1716 and z = s^2 < 0.0295, from the odd Taylor
// series 2 s (1 + z/3 + z^2/5 + ... + z^9/19) (the first omitted term,
// z^10/21, is below 2.3e-17 of the sum: a fifth of an ulp); e ln 2 is added
// in two parts, ln2_hi carrying 32
// significant bits so that e ln2_hi is exact for |e| < 2^21.  m - 1 is exact
// (Sterbenz), s is correctly rounded up to the rounding of m + 1, and the
// remaining operations add half an ulp each.  About 35 operations against
// ~105 of the library logarithm, which is correctly rounded.
CDI_HD double cdi_log(double x) {
  constexpr double kSqrtHalf = 0.70710678118654752440;
  constexpr double kLn2Hi = 0x1.62e42fee00000p-1;   // ln 2 to 32 significant bits
  constexpr double kLn2Lo = 0x1.a39ef35793c76p-33;  // ln 2 - kLn2Hi
  int e = 0;
  double m = __builtin_frexp(x, &e);   // x = m 2^e, m in [1/2, 1)
  if (m < kSqrtHalf) {
    m = 2.0 * m;
    e -= 1;
  }
  const double s = (m - 1.0) / (m + 1.0);
  const double z = s * s;
  double p = 1.0 / 19.0;
  p = __builtin_fma(p, z, 1.0 / 17.0);
  p = __builtin_fma(p, z, 1.0 / 15.0);
  p = __builtin_fma(p, z, 1.0 / 13.0);
  p = __builtin_fma(p, z, 1.0 / 11.0);
  p = __builtin_fma(p, z, 1.0 / 9.0);
  p = __builtin_fma(p, z, 1.0 / 7.0);
  p = __builtin_fma(p, z, 1.0 / 5.0);
  p = __builtin_fma(p, z, 1.0 / 3.0);
  const double t = 2.0 * s;
  const double tz = t * z;
  const double lm = __builtin_fma(tz, p, t);
  const double de = (double)e;
  return __builtin_fma(de, kLn2Hi, __builtin_fma(de, kLn2Lo, lm));
}

}  // namespace cdi
