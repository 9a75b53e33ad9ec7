// Device math shared by the kernels of libbumbar.
#pragma once

#include <hip/hip_runtime.h>

namespace bumbar {

// exp(x) for x <= 0 in double precision: Cody-Waite reduction x = k ln2 + r
// (ln 2 split into a 32-bit head, so k * head is exact, and a tail), then the
// degree-12 Taylor polynomial of e^r on |r| <= ln2/2, whose truncation error
// is below 2e-16 relative; the result is scaled by 2^k with ldexp. x is first
// clamped at -1000, where 2^k underflows to exactly 0, so x = -inf gives 0
// without a separate select. A NaN x also gives 0 (max ignores a NaN
// operand): callers that must reject NaN inputs detect them separately.
__device__ __forceinline__ double exp_nonpos(double x) {
  x = __builtin_fmax(x, -1000.0);
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
  return __builtin_ldexp(p, (int)kf);
}

// 1/x for a positive normal x: hardware reciprocal estimate refined by two
// Newton-Raphson steps (error about 1 ulp). Lighter on registers than the
// IEEE division sequence.
__device__ __forceinline__ double rcp_nr(double x) {
  double y = __builtin_amdgcn_rcp(x);
  double e = __builtin_fma(-x, y, 1.0);
  y = __builtin_fma(y, e, y);
  e = __builtin_fma(-x, y, 1.0);
  return __builtin_fma(y, e, y);
}

// ln(x) for 1 <= x <= 2^1000 (column sums of the sweep lie in [1, K]): a
// single-precision estimate y0 = log2f(x) ln 2 (relative error ~1e-7) refined
// by two Newton steps on exp, y <- y + x exp(-y) - 1, each squaring the error
// (1e-7 -> 1e-14 -> below double rounding). It reuses the exp above, so it
// needs no polynomial constants of its own (they would compete for scalar
// registers with the exp's coefficients inside the sweep kernels).
__device__ __forceinline__ double log_ge1(double x) {
  double y = (double)__builtin_amdgcn_logf((float)x) * 0.6931471805599453;
  y = y + __builtin_fma(x, exp_nonpos(-y), -1.0);
  y = y + __builtin_fma(x, exp_nonpos(-y), -1.0);
  return y;
}

}  // namespace bumbar
