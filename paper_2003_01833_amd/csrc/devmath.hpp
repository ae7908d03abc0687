// Device math for the kernel evaluations: exp on non-positive arguments and the
// reciprocal square root, in FP64, without the special-case handling that the
// general library routines carry (inputs here are finite, exp arguments lie in
// [-745, 0], and square roots are taken of positive squared distances).
#pragma once

#include <hip/hip_runtime.h>

namespace tagi {

constexpr double kLog2e = 0x1.71547652b82fep+0;  // log2(e)
constexpr double kLn2 = 0x1.62e42fefa39efp-1;    // ln(2)

// exp(v c) for finite v c <= 0, given cl2 = c log2(e) (the kernels scale their
// decay constants once): exp(v c) = 2^(v cl2) = 2^k 2^f with k the nearest
// integer to v cl2 and f = v cl2 - k, formed in one fused multiply-add from the
// same product (|f| <= 1/2, rounded once); 2^f by the degree-9 polynomial that
// interpolates 2^f at the 10 Chebyshev points of [-1/2, 1/2] (coefficients
// computed in 60-digit arithmetic by gen_exp_coeffs.py beside this file and
// rounded to double; relative error of the Horner evaluation at most 1.9e-14 on
// the interval, far below the treecode's own error). Rounding cl2 adds a
// relative error of at most |v c| 3.4e-16 (1.6e-14 for results above 1e-20).
// The nearest integer is formed by adding 1.5 * 2^52, whose ulp is 1, so the
// low word of the sum holds k in two's complement.
__device__ __forceinline__ double exp2_scaled(double v, double cl2) {
  constexpr double kShift = 0x1.8p52;
  const double t = __builtin_fma(v, cl2, kShift);
  const double kd = t - kShift;
  const int k = (int)__double2loint(t);
  const double f = __builtin_fma(v, cl2, -kd);
  double p = 0x1.b6571de2f2351p-24;
  p = __builtin_fma(p, f, 0x1.63ef969a64d3cp-20);
  p = __builtin_fma(p, f, 0x1.ffcb76789860fp-17);
  p = __builtin_fma(p, f, 0x1.43088e257f341p-13);
  p = __builtin_fma(p, f, 0x1.5d87fe908f88ap-10);
  p = __builtin_fma(p, f, 0x1.3b2ab72b175eep-7);
  p = __builtin_fma(p, f, 0x1.c6b08d7044119p-5);
  p = __builtin_fma(p, f, 0x1.ebfbdff8149f2p-3);
  p = __builtin_fma(p, f, 0x1.62e42fefa39f7p-1);
  p = __builtin_fma(p, f, 0x1.000000000003dp+0);
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

// 2/sqrt(x) for finite x > 0: the same Newton step written as
// 2 y' = y (3 - x y^2) with h = x y, three operations instead of four; callers
// that sum many such terms apply the factor 1/2 once to the sums (exact).
__device__ __forceinline__ double rsqrt_pos_x2(double x) {
  const double y = __builtin_amdgcn_rsq(x);
  const double h = x * y;
  return y * __builtin_fma(-h, y, 3.0);
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

// 2/sqrt(x) and 2 sqrt(x) from the step of rsqrt_pos_x2: e = 3 - h y,
// 2 y' = y e, 2 sqrt(x) = h e.
__device__ __forceinline__ void rsqrt_sqrt_x2(double x, double& rinv2, double& r2) {
  const double y = __builtin_amdgcn_rsq(x);
  const double h = x * y;
  const double e = __builtin_fma(-h, y, 3.0);
  rinv2 = y * e;
  r2 = h * e;
}

}  // namespace tagi
