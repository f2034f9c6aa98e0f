// Spin-weighted spherical harmonics -2Y_lm(theta, phi) on the device: the
// angular functions of Eq. main_wave for a Schwarzschild inspiral (the
// spheroidal harmonics reduce to spherical ones, Sec. 2.1), from the
// Goldberg explicit sum
//   sY_lm = (-1)^m sqrt[(l+m)!(l-m)!(2l+1) / (4 pi (l+s)!(l-s)!)]
//           sum_r C(l-s,r) C(l+s,r+s-m) (-1)^(l-r-s) sin(th/2)^(2l-k) cos(th/2)^k e^{i m phi},
// k = 2r+s-m, and its theta derivative term by term.  Binomial coefficients
// come from an exact table (every entry below 2^53), integer powers from
// repeated squaring.
#pragma once

#include "fdemri_internal.hpp"

namespace fdemri {

// C(n, k) for 0 <= k <= n <= kBinomN - 1 (n = l - s <= FDEMRI_MAX_L + 2).
constexpr int kBinomN = kMaxL + 3;

struct BinomTable {
  double v[kBinomN][kBinomN];
  constexpr BinomTable() : v() {
    for (int n = 0; n < kBinomN; ++n) {
      v[n][0] = 1.0;
      for (int k = 1; k <= n; ++k) v[n][k] = v[n - 1][k - 1] + (k < n ? v[n - 1][k] : 0.0);
    }
  }
};

__device__ __constant__ const BinomTable kBinom{};

__device__ __forceinline__ double ipow(double x, int e) {
  double r = 1.0;
  while (e > 0) {
    if (e & 1) r *= x;
    x *= x;
    e >>= 1;
  }
  return r;
}

// (-1)^m sqrt[(l+m)!(l-m)!(2l+1) / (4 pi (l+s)!(l-s)!)] for s = -2.
__device__ __forceinline__ double goldberg_pref(int l, int m) {
  const int s = -2;
  if (l < 2 || l > kMaxL || m > l || m < -l) return 0.0;  // no harmonic (such rows are flagged)
  double ratio = 1.0;
  int a = l + m, b = l - s;
  if (a >= b)
    for (int j = b + 1; j <= a; ++j) ratio *= (double)j;
  else
    for (int j = a + 1; j <= b; ++j) ratio /= (double)j;
  a = l - m;
  b = l + s;
  if (a >= b)
    for (int j = b + 1; j <= a; ++j) ratio *= (double)j;
  else
    for (int j = a + 1; j <= b; ++j) ratio /= (double)j;
  return ((m & 1) ? -1.0 : 1.0) * sqrt(ratio * (2 * l + 1) / (4.0 * kPi));
}

// Term r of the Goldberg sum (s = -2) and, in dterm, its theta derivative.
__device__ __forceinline__ double goldberg_term(int l, int m, int r, double sh, double ch, double* dterm) {
  const int s = -2;
  const int b2 = r + s - m;
  if (dterm) *dterm = 0.0;
  if (l < 2 || l > kMaxL) return 0.0;  // outside the binomial table (such rows are flagged)
  if (r < 0 || r > l - s || b2 < 0 || b2 > l + s) return 0.0;
  const int k = 2 * r + s - m;
  const int ea = 2 * l - k;
  const double coef = (((l - r - s) & 1) ? -1.0 : 1.0) * kBinom.v[l - s][r] * kBinom.v[l + s][b2];
  const double pe = ipow(sh, ea), pk = ipow(ch, k);
  if (dterm) {
    double dt = 0.0;
    if (ea > 0) dt += 0.5 * ea * ipow(sh, ea - 1) * (pk * ch);
    if (k > 0) dt -= 0.5 * k * (pe * sh) * ipow(ch, k - 1);
    *dterm = coef * dt;
  }
  return coef * pe * pk;
}

// Y (x, y) and dY/dtheta (z, w) for s = -2, by one thread.
__device__ inline double4 swsh_m2_with_dtheta(int l, int m, double theta, double phi) {
  const double sh = sin(0.5 * theta), ch = cos(0.5 * theta);
  double acc = 0.0, dacc = 0.0;
  for (int r = 0; r <= l + 2; ++r) {
    double dt;
    acc += goldberg_term(l, m, r, sh, ch, &dt);
    dacc += dt;
  }
  const double pref = goldberg_pref(l, m);
  double sp, cp;
  sincos((double)m * phi, &sp, &cp);
  return make_double4(pref * acc * cp, pref * acc * sp, pref * dacc * cp, pref * dacc * sp);
}

// Y_{l,m} (x, y) and Y_{l,-m} (z, w) for s = -2, by a whole wavefront: each
// half-wave sums the terms of one of the two harmonics, one term per lane.
// Every lane returns both.
__device__ inline double4 swsh_m2_pair_wave(int l, int m, double theta, double phi) {
  const int lane = threadIdx.x & 63;
  const int mm = (lane < 32) ? m : -m;
  const double sh = sin(0.5 * theta), ch = cos(0.5 * theta);
  double part = 0.0;
  for (int r = lane & 31; r <= l + 2; r += 32) part += goldberg_term(l, mm, r, sh, ch, nullptr);
#pragma unroll
  for (int off = 16; off >= 1; off >>= 1) part += __shfl_xor(part, off, 64);
  const double pref = goldberg_pref(l, mm);
  const double sum_p = __shfl(part, 0, 64), sum_m = __shfl(part, 32, 64);
  const double pref_p = __shfl(pref, 0, 64), pref_m = __shfl(pref, 32, 64);
  double sp, cp;
  sincos((double)m * phi, &sp, &cp);
  return make_double4(pref_p * sum_p * cp, pref_p * sum_p * sp, pref_m * sum_m * cp, -pref_m * sum_m * sp);
}

}  // namespace fdemri
