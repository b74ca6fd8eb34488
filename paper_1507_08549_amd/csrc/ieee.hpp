// ieee.hpp -- correctly rounded FP64 division and square root on the device.
//
// The compiler's FP64 division is a reciprocal refined by Newton steps and a
// final fused correction; its result is within one unit in the last place but
// not always the correctly rounded one: quotients that fall within a tiny
// fraction of an ulp of a halfway point between two doubles can be rounded to
// the wrong side (0x1.6666666666663p-2 / 0x1.ffffffffffffbp-4 is one).  The
// bit-exact paths need IEEE results, so every FP64 division and square root
// on them goes through the helpers below: take the hardware result q, then
// compare it with its neighbour on the side of the true result.  Both are
// faithful roundings, so the residuals a - q b and a - q' b (x - s^2 for the
// root) are exact in one fma each, and the one with the smaller residual is
// the correctly rounded result (a quotient or root of doubles is never
// exactly halfway between two doubles, so there are no ties).
#pragma once
#include <hip/hip_runtime.h>

namespace hy {

// q and its neighbour one ulp away from or towards zero: away when the sign
// of dir matches the sign of q (compared on the high words' sign bits).  A
// neighbour that is not a finite double of the same sign (from 0 or the
// largest double) only ever loses the comparison below.
__device__ __forceinline__ double ieee_step(double q, double dir) {
  const long long bq = __double_as_longlong(q);
  const int hi = (int)((unsigned long long)bq >> 32) ^ (int)((unsigned long long)__double_as_longlong(dir) >> 32);
  return __longlong_as_double(bq + (hi < 0 ? -1LL : 1LL));
}

// No branches: where t = 0 (exact), q = 0, or q is not finite, the residual of
// the neighbour is never smaller, so q stays.
__device__ __forceinline__ double cr_div(double a, double b) {
  const double q = a / b;
  const double t = __builtin_fma(-q, b, a);
  // the true quotient q + t/b lies on the side of sign(t) sign(b)
  const double q2 = ieee_step(q, __builtin_copysign(1.0, t) * b);
  const double t2 = __builtin_fma(-q2, b, a);
  return __builtin_fabs(t2) < __builtin_fabs(t) ? q2 : q;
}

// cr_div for a positive normal denominator whose reciprocal is normal and a
// quotient that is zero or normal: a faithful quotient from the hardware
// reciprocal, one Newton step and one correction step (q0 = a r,
// q = q0 + (a - q0 b) r), without the scaling and special-value steps of the
// general division sequence, then the same neighbour check (with b > 0 the
// true quotient lies on the side of sign(t) alone).  With r = (1 + d) / b
// after the Newton step, q0 = Q (1 + D) with D = d + (rounding of a r), and
// the correction leaves Q (1 - D (d + e)) before its rounding (e: rounding of
// the residual), so the relative error before the last rounding is about
// d^2: the hardware reciprocal's error (measured at most 2^-24.4) is squared
// twice, far below half an ulp.  The WENO face values are such quotients:
// their denominators, products of sums of weights, lie between about 3e-47
// (eps = 1e-6) and the overflow of the numerator that comes with them.
__device__ __forceinline__ double cr_div_pos_normal(double a, double b) {
  double r = __builtin_amdgcn_rcp(b);
  r = __builtin_fma(r, __builtin_fma(-b, r, 1.0), r);
  const double q0 = a * r;
  const double q = __builtin_fma(__builtin_fma(-q0, b, a), r, q0);
  const double t = __builtin_fma(-q, b, a);
  const double q2 = ieee_step(q, t);
  const double t2 = __builtin_fma(-q2, b, a);
  return __builtin_fabs(t2) < __builtin_fabs(t) ? q2 : q;
}

// Correctly rounded 1 / b for a positive normal b with a normal reciprocal
// (densities, radii): the hardware reciprocal refined by two Newton steps is
// faithful, then the neighbour check.  (Other b: not correctly rounded; the
// states where that happens are reported as unphysical anyway.)
__device__ __forceinline__ double cr_rcp_pos(double b) {
  double r = __builtin_amdgcn_rcp(b);
  r = __builtin_fma(r, __builtin_fma(-b, r, 1.0), r);
  r = __builtin_fma(r, __builtin_fma(-b, r, 1.0), r);
  const double t = __builtin_fma(-r, b, 1.0);
  const double r2 = ieee_step(r, t);
  const double t2 = __builtin_fma(-r2, b, 1.0);
  return __builtin_fabs(t2) < __builtin_fabs(t) ? r2 : r;
}

__device__ __forceinline__ double cr_sqrt(double x) {
  const double s = __builtin_sqrt(x);
  const double t = __builtin_fma(-s, s, x);
  const double s2 = ieee_step(s, t);
  const double t2 = __builtin_fma(-s2, s2, x);
  return __builtin_fabs(t2) < __builtin_fabs(t) ? s2 : s;
}

// Correctly rounded square root of a positive normal x (squared sound
// speeds): reciprocal square root, Goldschmidt refinement (g -> sqrt(x),
// h -> 1 / (2 sqrt(x))) and two corrections, then the neighbour check; no
// scaling or special-value steps.  (x <= 0 gives NaN, not the IEEE 0: such a
// state is reported as unphysical anyway.)
__device__ __forceinline__ double cr_sqrt_pos(double x) {
  const double y = __builtin_amdgcn_rsq(x);
  double g = x * y, h = 0.5 * y;
  const double e = __builtin_fma(-h, g, 0.5);
  g = __builtin_fma(g, e, g);
  h = __builtin_fma(h, e, h);
  g = __builtin_fma(__builtin_fma(-g, g, x), h, g);
  const double s = __builtin_fma(__builtin_fma(-g, g, x), h, g);
  const double t = __builtin_fma(-s, s, x);
  const double s2 = ieee_step(s, t);
  const double t2 = __builtin_fma(-s2, s2, x);
  return __builtin_fabs(t2) < __builtin_fabs(t) ? s2 : s;
}

}  // namespace hy
