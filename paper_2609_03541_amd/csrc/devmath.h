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


// exp(x) for x <= 0 with a 64-entry table: x = (64 q + j) ln2/64 + r with
// |r| <= ln2/128, e^x = 2^q 2^(j/64) e^r, e^r by its degree-5 Taylor
// polynomial (truncation below 4e-17 relative on that interval). tab holds
// 2^(j/64), j = 0..63, each correctly rounded (kExp2Frac64 below, computed
// from the definition in 60-digit decimal arithmetic); kernels stage it in
// LDS. ln2/64 is split into a 32-bit head (k * head exact for the clamped
// range) and a tail. Same clamp and NaN behaviour as exp_nonpos; about 13
// FP64 operations instead of 18, plus one LDS read.
__device__ __forceinline__ double exp_nonpos_tab(double x, const double* __restrict__ tab) {
  x = __builtin_fmax(x, -1000.0);
  // round x 64/ln2 to an integer by adding 1.5 2^52 (|x 64/ln2| < 2^17 here):
  // the sum's low 32 bits are that integer in two's complement
  const double big = __builtin_fma(x, 92.33248261689366, 6755399441055744.0);
  const int ki = (int)(uint32_t)__builtin_bit_cast(unsigned long long, big);
  const double kf = big - 6755399441055744.0;
  double r = __builtin_fma(kf, -0.010830424696905538, x);
  r = __builtin_fma(kf, 6.563929801064195e-13, r);
  double p = __builtin_fma(r, 0.008333333333333333, 0.041666666666666664);
  p = __builtin_fma(p, r, 0.16666666666666666);
  p = __builtin_fma(p, r, 0.5);
  p = __builtin_fma(p, r, 1.0);
  p = __builtin_fma(p, r, 1.0);
  return __builtin_ldexp(tab[ki & 63] * p, ki >> 6);
}

// 2^(j/64), j = 0..63, correctly rounded.
static __constant__ const double kExp2Frac64[64] = {
    1.0, 1.0108892860517005, 1.0218971486541166, 1.0330248790212284,
    1.0442737824274138, 1.0556451783605572, 1.0671404006768237, 1.0787607977571199,
    1.0905077326652577, 1.102382583307841, 1.1143867425958924, 1.1265216186082418,
    1.1387886347566916, 1.1511892299529827, 1.1637248587775775, 1.1763969916502812,
    1.189207115002721, 1.202156731452703, 1.215247359980469, 1.22848053610687,
    1.241857812073484, 1.255380757024691, 1.2690509571917332, 1.2828700160787783,
    1.2968395546510096, 1.3109612115247644, 1.3252366431597413, 1.339667524053303,
    1.3542555469368927, 1.3690024229745905, 1.383909881963832, 1.3989796725383112,
    1.4142135623730951, 1.42961333839197, 1.4451808069770467, 1.460917794180647,
    1.4768261459394993, 1.4929077282912648, 1.5091644275934228, 1.5255981507445384,
    1.5422108254079407, 1.559004400237837, 1.5759808451078865, 1.593142151342267,
    1.6104903319492543, 1.6280274218573478, 1.645755478153965, 1.6636765803267364,
    1.681792830507429, 1.7001063537185235, 1.718619298122478, 1.7373338352737062,
    1.7562521603732995, 1.7753764925265212, 1.7947090750031072, 1.8142521755003989,
    1.8340080864093424, 1.8539791250833855, 1.8741676341103, 1.8945759815869656,
    1.9152065613971474, 1.9360617934922943, 1.9571441241754002, 1.978456026387951,
};

}  // namespace bumbar
