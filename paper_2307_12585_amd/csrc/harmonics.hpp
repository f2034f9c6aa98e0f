// Spin-weighted spherical harmonics -2Y_lm(theta, phi) on the device: the
// angular functions of Eq. main_wave for a Schwarzschild inspiral (the
// spheroidal harmonics reduce to spherical ones, Sec. 2.1), from the
// Goldberg explicit sum
//   sY_lm = (-1)^m sqrt[(l+m)!(l-m)!(2l+1) / (4 pi (l+s)!(l-s)!)]
//           sum_r C(l-s,r) C(l+s,r+s-m) (-1)^(l-r-s) sin(th/2)^(2l-k) cos(th/2)^k e^{i m phi},
// k = 2r+s-m, and its theta derivative term by term.
#pragma once

#include "fdemri_internal.hpp"

namespace fdemri {

// returns Y (x, y) and dY/dtheta (z, w) for s = -2
__device__ inline double4 swsh_m2_with_dtheta(int l, int m, double theta, double phi) {
  const int s = -2;
  double ratio = 1.0;  // (l+m)!(l-m)! / ((l+s)!(l-s)!)
  {
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
  }
  const double pref = ((m & 1) ? -1.0 : 1.0) * sqrt(ratio * (2 * l + 1) / (4.0 * kPi));
  const double sh = sin(0.5 * theta), ch = cos(0.5 * theta);
  double acc = 0.0, dacc = 0.0;
  for (int r = 0; r <= l - s; ++r) {
    const int b2 = r + s - m;
    if (b2 < 0 || b2 > l + s) continue;
    long long c1 = 1, c2 = 1;  // C(l-s, r), C(l+s, b2): exact for l <= 40
    for (int j = 1; j <= r; ++j) c1 = c1 * (l - s - r + j) / j;
    for (int j = 1; j <= b2; ++j) c2 = c2 * (l + s - b2 + j) / j;
    const int k = 2 * r + s - m;
    const int ea = 2 * l - k;
    const double coef = (((l - r - s) & 1) ? -1.0 : 1.0) * (double)c1 * (double)c2;
    acc += coef * pow(sh, (double)ea) * pow(ch, (double)k);
    double dt = 0.0;
    if (ea > 0) dt += 0.5 * ea * pow(sh, (double)(ea - 1)) * pow(ch, (double)(k + 1));
    if (k > 0) dt -= 0.5 * k * pow(sh, (double)(ea + 1)) * pow(ch, (double)(k - 1));
    dacc += coef * dt;
  }
  double sp, cp;
  sincos((double)m * phi, &sp, &cp);
  return make_double4(pref * acc * cp, pref * acc * sp, pref * dacc * cp, pref * dacc * sp);
}

__device__ inline double2 swsh_m2(int l, int m, double theta, double phi) {
  const double4 v = swsh_m2_with_dtheta(l, m, theta, phi);
  return make_double2(v.x, v.y);
}

}  // namespace fdemri
