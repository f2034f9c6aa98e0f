// Per-root factor of the third-order stationary-phase term (Sec. 2.2,
// Eq. extendedspa1) on the device.
//
// For a root with local derivatives gd = d|F|/dt, gdd = d2|F|/dt2 the
// factor multiplying H(t_j) e^{i[2 pi f t_j - Phi(t_j)]} is
//   G = |gd|^{-1/2} e^{-i pi/4 sgn gd} W(X),   X = 2 pi gd^3 / (3 gdd^2),
//   W(X) = sqrt(2|X|/pi) e^{-i pi/4 sgn X} e^{-iX} K_{1/3}(-iX)
// (the printed constant of Eq. extendedspa1 is taken with the opposite sign,
// the reading under which the formula reduces to the standard SPA as
// gdd -> 0 as the paper states).  Evaluation:
//  * gdd = 0: W = 1;
//  * |X| >= X_B: W = sum_k a_k (i/X)^k (large-argument expansion of the
//    exponentially scaled K_{1/3});
//  * |X| <  X_B: the same factor in Airy form,
//      G = pi (pi|gdd|)^{-1/3} Q(y)  (conjugated when sgn gd < 0),
//      Q(y) = [Ai(-y^2) - i Bi(-y^2)] e^{-i 2y^3/3},  y = (3|X|/2)^{1/3},
//    from piecewise Chebyshev tables; it is finite at gd = 0, where the
//    sign is the direction of the monotonic piece.
// The paper approximates the same function by two polynomial fits with
// ~1e-3 relative error; these tables hold it to FP64 (FP32) accuracy.
#pragma once

#include "fdemri_internal.hpp"
#include "w_table.inc"

namespace fdemri {

__device__ __forceinline__ double2 q_cheb64(double y) {
  constexpr double w = FDW_Y_B / FDW_NINT;
  int j = (int)(y * (FDW_NINT / FDW_Y_B));
  j = j < 0 ? 0 : (j > FDW_NINT - 1 ? FDW_NINT - 1 : j);
  const double x = 2.0 * (y - j * w) / w - 1.0;
  const double* cr = fdw_q64_re + j * (FDW_DEG64 + 1);
  const double* ci = fdw_q64_im + j * (FDW_DEG64 + 1);
  double b1r = 0.0, b2r = 0.0, b1i = 0.0, b2i = 0.0;
  const double x2 = 2.0 * x;
  // kept rolled: the branch is rare, and unrolling would hold every
  // coefficient in registers at once
#pragma unroll 1
  for (int k = FDW_DEG64; k >= 1; --k) {
    const double tr = x2 * b1r - b2r + cr[k];
    const double ti = x2 * b1i - b2i + ci[k];
    b2r = b1r;
    b1r = tr;
    b2i = b1i;
    b1i = ti;
  }
  return make_double2(x * b1r - b2r + cr[0], x * b1i - b2i + ci[0]);
}

__device__ __forceinline__ float2 q_cheb32(float y) {
  constexpr float w = (float)(FDW_Y_B / FDW_NINT);
  int j = (int)(y * (float)(FDW_NINT / FDW_Y_B));
  j = j < 0 ? 0 : (j > FDW_NINT - 1 ? FDW_NINT - 1 : j);
  const float x = 2.0f * (y - j * w) / w - 1.0f;
  const float* cr = fdw_q32_re + j * (FDW_DEG32 + 1);
  const float* ci = fdw_q32_im + j * (FDW_DEG32 + 1);
  float b1r = 0.f, b2r = 0.f, b1i = 0.f, b2i = 0.f;
  const float x2 = 2.0f * x;
#pragma unroll 1
  for (int k = FDW_DEG32; k >= 1; --k) {
    const float tr = x2 * b1r - b2r + cr[k];
    const float ti = x2 * b1i - b2i + ci[k];
    b2r = b1r;
    b1r = tr;
    b2i = b1i;
    b1i = ti;
  }
  return make_float2(x * b1r - b2r + cr[0], x * b1i - b2i + ci[0]);
}

// Even and odd parts of the large-argument series in v = u^2: the sums over
// j <= J of (-1)^j a_{2j} v^j and (-1)^j a_{2j+1} v^j (Horner, highest term
// first).
template <int J>
__device__ __forceinline__ double asym_even(double v) {
  double s = (J & 1) ? -fdw_asym64[2 * J] : fdw_asym64[2 * J];
#pragma unroll
  for (int j = J - 1; j >= 0; --j) s = fma_sc(s, v, (j & 1) ? -fdw_asym64[2 * j] : fdw_asym64[2 * j]);
  return s;
}

template <int J>
__device__ __forceinline__ double asym_odd(double v) {
  double s = (J & 1) ? -fdw_asym64[2 * J + 1] : fdw_asym64[2 * J + 1];
#pragma unroll
  for (int j = J - 1; j >= 0; --j) s = fma_sc(s, v, (j & 1) ? -fdw_asym64[2 * j + 1] : fdw_asym64[2 * j + 1]);
  return s;
}

// G in FP64.  dir = direction of the piece (used only when gd == 0).
// |gd|^{-1/2} is formed once (refined hardware estimate) and also gives
// |u| = |1/X| = 3 gdd^2 / (2 pi |gd|^3) through its sixth power.  |u| <= 1/X_B
// selects the large-argument expansion, whose length is chosen per wave from
// the largest |u| among the active lanes (|u| <= 1e-5: terms to u^3, first
// omitted below 1e-21; |u| <= 1e-3: terms to u^7, below 1e-23; otherwise the
// full table).  gd == 0 (a root on a turning point) has no finite |u| and
// takes the Airy form, which is finite there.
__device__ __forceinline__ double2 spa_factor64(double gd, double gdd, int dir) {
  constexpr double kRsqrt2 = 0.70710678118654752440;
  constexpr double k3Over2Pi = 0.47746482927568600730;
  constexpr double k2PiOver3 = 2.0943951023931954923;
  const double agd = fabs(gd);
  const double rs = rsq_nr2(agd);
  const double rs2 = rs * rs;
  // gdd = 0 gives |u| = 0, the standard SPA, with no special case; gd = 0
  // leaves no finite |u| and takes the Airy form
  const double au = k3Over2Pi * gdd * gdd * (rs2 * rs2 * rs2);
  if (gd != 0.0 && au <= 1.0 / FDW_X_B) {
    // W = re + i sg im with re, im the even and odd parts of the series in
    // |u| (u = 1/X carries the sign sg of gd); then
    // G = c (1 - i sg) W = c (re + im) + i sg c (im - re), the factor sg
    // applied by giving c the sign of gd.
    const double v = au * au;
    double re, im;
    if (__all(au <= 1e-5)) {
      re = asym_even<1>(v);
      im = asym_odd<1>(v);
    } else if (__all(au <= 1e-3)) {
      re = asym_even<3>(v);
      im = asym_odd<3>(v);
    } else {
      re = asym_even<(FDW_NASYM64 - 1) / 2>(v);
      im = asym_odd<(FDW_NASYM64 - 2) / 2>(v);
    }
    im *= au;
    const double c = kRsqrt2 * rs;
    return make_double2(c * (re + im), __builtin_copysign(c, gd) * (im - re));
  }
  if (gdd == 0.0) {
    // reached only when |u| above could not be formed (gd = 0, or |gd| so
    // small that rs^6 overflows): W = 1, or no contribution when gd = 0 too
    if (gd == 0.0) return make_double2(0.0, 0.0);
    const double c = kRsqrt2 * rs;
    return make_double2(c, -__builtin_copysign(c, gd));
  }
  const int sg = gd > 0.0 ? 1 : (gd < 0.0 ? -1 : dir);
  const double ax = k2PiOver3 * agd * agd * agd * rcp_nr2(gdd * gdd);  // |X|
  const double y = cbrt(1.5 * ax);
  double2 q = q_cheb64(y);
  if (sg < 0) q.y = -q.y;
  const double pref = kPi / cbrt(kPi * fabs(gdd));
  return make_double2(pref * q.x, pref * q.y);
}

// G in FP32 from FP64 derivatives (the mixed-precision path keeps gd, gdd in
// FP64 and evaluates the special function in FP32); same branches as the
// FP64 factor.
__device__ __forceinline__ float2 spa_factor32(double gd, double gdd, int dir) {
  constexpr float kRsqrt2 = 0.70710678118654752440f;
  constexpr double k3Over2Pi = 0.47746482927568600730;
  constexpr double k2PiOver3 = 2.0943951023931954923;
  const double agd = fabs(gd);
  const double au = k3Over2Pi * gdd * gdd * rcp_nr1(agd * agd * agd);
  if (gd != 0.0 && au <= 1.0 / FDW_X_B) {
    const float uf = (float)au;
    const float v = uf * uf;
    float re, im;
    if (__all(au <= 1e-3)) {
      // every active lane has |u| <= 1e-3: terms to u^3 (the first omitted
      // one, a_4 u^4, is below 1e-13)
      re = __builtin_fmaf(-fdw_asym32[2], v, fdw_asym32[0]);
      im = __builtin_fmaf(-fdw_asym32[3], v, fdw_asym32[1]);
    } else {
      re = 0.f;
      im = 0.f;
#pragma unroll
      for (int j = (FDW_NASYM32 - 1) / 2; j >= 0; --j) {
        const float sgn = (j & 1) ? -1.f : 1.f;
        re = re * v + sgn * fdw_asym32[2 * j];
        if (2 * j + 1 < FDW_NASYM32) im = im * v + sgn * fdw_asym32[2 * j + 1];
      }
    }
    im *= uf;
    const float c = kRsqrt2 * rsqrtf((float)agd);
    return make_float2(c * (re + im), __builtin_copysignf(c, (float)gd) * (im - re));
  }
  if (gdd == 0.0) {
    // as in the FP64 factor: W = 1, or nothing when gd = 0 too
    if (gd == 0.0) return make_float2(0.f, 0.f);
    const float c = (float)(kRsqrt2 * rsq_nr2(agd));
    return make_float2(c, -__builtin_copysignf(c, (float)gd));
  }
  const int sg = gd > 0.0 ? 1 : (gd < 0.0 ? -1 : dir);
  const float y = cbrtf((float)(1.5 * k2PiOver3 * agd * agd * agd * rcp_nr2(gdd * gdd)));
  float2 q = q_cheb32(y);
  if (sg < 0) q.y = -q.y;
  const float pref = (float)(kPi / cbrt(kPi * fabs(gdd)));
  return make_float2(pref * q.x, pref * q.y);
}

}  // namespace fdemri
