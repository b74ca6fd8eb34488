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

__device__ __forceinline__ double ieee_next_toward(double q, bool up) {
  long long b = __double_as_longlong(q);
  b += ((q > 0.0) == up) ? 1 : -1;
  return __longlong_as_double(b);
}

__device__ __forceinline__ double cr_div(double a, double b) {
  double q = a / b;
  const double t = __builtin_fma(-q, b, a);
  if (t != 0.0 && q != 0.0 && __builtin_isfinite(q)) {
    const bool up = (t > 0.0) == (b > 0.0);  // a/b lies above q
    const double q2 = ieee_next_toward(q, up);
    const double t2 = __builtin_fma(-q2, b, a);
    if (__builtin_fabs(t2) < __builtin_fabs(t)) q = q2;
  }
  return q;
}

__device__ __forceinline__ double cr_sqrt(double x) {
  double s = __builtin_sqrt(x);
  const double t = __builtin_fma(-s, s, x);
  if (t != 0.0 && s > 0.0 && __builtin_isfinite(s)) {
    const double s2 = ieee_next_toward(s, t > 0.0);
    const double t2 = __builtin_fma(-s2, s2, x);
    if (__builtin_fabs(t2) < __builtin_fabs(t)) s = s2;
  }
  return s;
}

}  // namespace hy
