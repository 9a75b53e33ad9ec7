// Device math shared by the kernels of libbumbar.
#pragma once

#include <hip/hip_runtime.h>

namespace bumbar {

// exp(x) for x <= 0 in double precision: Cody-Waite reduction x = k ln2 + r
// (ln 2 split into a 32-bit head, so k * head is exact, and a tail), then the
// degree-12 Taylor polynomial of e^r on |r| <= ln2/2, whose truncation error
// is below 2e-16 relative; the result is scaled by 2^k with ldexp. Returns
// exactly 0 for x < -708 (and for x = -inf); NaN propagates.
__device__ __forceinline__ double exp_nonpos(double x) {
  const double kf = __builtin_rint(x * 1.4426950408889634);
  double r = __builtin_fma(kf, -0.6931471803691238, x);
  r = __builtin_fma(kf, -1.9082149292705877e-10, r);
  double p = 2.08767569878681e-09;
  p = __builtin_fma(p, r, 2.505210838544172e-08);
  p = __builtin_fma(p, r, 2.755731922398589e-07);
  p = __builtin_fma(p, r, 2.7557319223985893e-06);
  p = __builtin_fma(p, r, 2.48015873015873e-05);
  p = __builtin_fma(p, r, 0.0001984126984126984);
  p = __builtin_fma(p, r, 0.001388888888888889);
  p = __builtin_fma(p, r, 0.008333333333333333);
  p = __builtin_fma(p, r, 0.041666666666666664);
  p = __builtin_fma(p, r, 0.16666666666666666);
  p = __builtin_fma(p, r, 0.5);
  p = __builtin_fma(p, r, 1.0);
  p = __builtin_fma(p, r, 1.0);
  const int ki = (int)__builtin_fmax(kf, -1100.0);
  const double y = __builtin_ldexp(p, ki);
  return (x < -708.0) ? 0.0 : y;
}

}  // namespace bumbar
