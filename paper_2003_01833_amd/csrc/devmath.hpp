// Device math for the kernel evaluations: exp on non-positive arguments and the
// reciprocal square root, in FP64, without the special-case handling that the
// general library routines carry (inputs here are finite, exp arguments lie in
// [-745, 0], and square roots are taken of positive squared distances).
#pragma once

#include <hip/hip_runtime.h>

namespace tagi {

// exp(x) for finite x <= 0. Cody and Waite's additive range reduction
// (W. J. Cody and W. Waite, Software Manual for the Elementary Functions, 1980):
// k = nearest integer to x / ln 2, r = x - k ln 2 in one fused multiply-add with
// ln 2 rounded to double (which adds at most |k| 2^-54 ln 2 to r: 1.6e-15 for
// exp(x) > 1e-20, 2.6e-14 at the underflow end), |r| <= ln(2)/2; then
// exp(r) by the degree-9 polynomial that interpolates exp at the 10 Chebyshev
// points of [-ln 2 / 2, ln 2 / 2] (coefficients computed in 60-digit arithmetic
// by gen_exp_coeffs.py beside this file and rounded to double; relative error of
// the Horner evaluation at most 1.9e-14 on the interval, far below the
// treecode's own error), and exp(x) = 2^k exp(r).
// The nearest integer is formed by adding 1.5 * 2^52, whose ulp is 1, so the
// low word of the sum holds k in two's complement.
__device__ __forceinline__ double exp_nonpos(double x) {
  constexpr double kLog2e = 0x1.71547652b82fep+0;
  constexpr double kShift = 0x1.8p52;
  constexpr double kLn2 = 0x1.62e42fefa39efp-1;
  const double t = __builtin_fma(x, kLog2e, kShift);
  const double kd = t - kShift;
  const int k = (int)__double2loint(t);
  const double r = __builtin_fma(kd, -kLn2, x);
  double p = 0x1.72e107c874de9p-19;
  p = __builtin_fma(p, r, 0x1.a17df0d914d6cp-16);
  p = __builtin_fma(p, r, 0x1.a01994c849582p-13);
  p = __builtin_fma(p, r, 0x1.6c162bb7d965cp-10);
  p = __builtin_fma(p, r, 0x1.11111123bf154p-7);
  p = __builtin_fma(p, r, 0x1.55555588b8403p-5);
  p = __builtin_fma(p, r, 0x1.5555555550d88p-3);
  p = __builtin_fma(p, r, 0x1.ffffffffe74f1p-2);
  p = __builtin_fma(p, r, 0x1.0000000000006p+0);
  p = __builtin_fma(p, r, 0x1.000000000003dp+0);
  return __builtin_amdgcn_ldexp(p, k);
}

// 1/sqrt(x) for finite x > 0: the hardware estimate y of v_rsq_f64 (relative
// error below 2^-24) refined by one Newton step, e = 1 - x y^2,
// y' = y + y e / 2, which squares the error (1.5 e^2 < 6e-15).
__device__ __forceinline__ double rsqrt_pos(double x) {
  const double y = __builtin_amdgcn_rsq(x);
  const double e = __builtin_fma(-x * y, y, 1.0);
  return __builtin_fma(y, 0.5 * e, y);
}

// 1/sqrt(x) and sqrt(x) for finite x > 0 from the same Newton step: with
// h = x y, sqrt(x) = x y' = h + h e / 2 (same error bound).
__device__ __forceinline__ void rsqrt_sqrt(double x, double& rinv, double& r) {
  const double y = __builtin_amdgcn_rsq(x);
  const double h = x * y;
  const double e2 = 0.5 * __builtin_fma(-h, y, 1.0);
  rinv = __builtin_fma(y, e2, y);
  r = __builtin_fma(h, e2, h);
}

}  // namespace tagi
