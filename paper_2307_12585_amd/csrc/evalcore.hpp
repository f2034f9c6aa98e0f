// Per-root arithmetic of the frequency-domain mode sum (Sec. 2.2), shared
// by the forward gather and the adjoint so that both evaluate bit-identical
// roots, phases and factors.
//
// For a voice (m, n) on a monotonic piece with sign s and direction d, and a
// bin f whose root lies in spline segment i (Eq. cubic_equation):
//   |F_V|(t_i + tau) = s (F0 + a1 tau + a2 tau^2 + a3 tau^3),
//   s Phi_V(t_i + tau) = s (Phi_V,i + b1 tau + b2 tau^2 + b3 tau^3),
// with F0 = m F_phi,i + n F_r,i from the knot data and a_k, b_k the
// mode-weighted spline coefficients of the fundamental frequencies and
// phases.
#pragma once

#include "spa.hpp"

namespace fdemri {

struct SegData {
  double ti, h, F0, F1;   // knot time, segment length, voice frequency at both knots
  double a1, a2, a3;      // frequency spline coefficients (mode-weighted)
  double b1, b2, b3;      // phase spline coefficients (mode-weighted)
  double Ppi, Pri;        // Phi_phi, Phi_r knot values at t_i
};

// Bracket of the root inside segment i of piece P: [tl, th] in tau, with
// |F_V| = gl, gh at its ends (piece end values at the piece's first/last
// segment, knot values elsewhere).
struct Bracket {
  double tl, th, gl, gh;
};

__device__ __forceinline__ Bracket make_bracket(const Piece& P, int i, double sd, const SegData& S) {
  const bool first = (i == P.seg_a), last = (i == P.seg_b);
  Bracket B;
  B.tl = first ? P.tau_a : 0.0;
  B.th = last ? P.tau_b : S.h;
  B.gl = first ? P.g_a : sd * S.F0;
  B.gh = last ? P.g_b : sd * S.F1;
  return B;
}

// Root of s (F0 + a1 tau + a2 tau^2 + a3 tau^3) = f on [tl, th] (|F_V|
// monotonic there with direction d): secant start, Newton steps safeguarded
// by bisection of the shrinking bracket.
__device__ __forceinline__ double solve_root(double f, double sd, double dd, const SegData& S, const Bracket& B) {
  double tau = B.tl;
  const double dg = B.gh - B.gl;
  if (dg != 0.0) tau = B.tl + (f - B.gl) * (B.th - B.tl) * rcp_nr1(dg);
  tau = fmin(fmax(tau, B.tl), B.th);
  double blo = B.tl, bhi = B.th;
  const double tol = 4e-16 * fmax(S.h, 1.0);
  for (int it = 0; it < 100; ++it) {
    const double r = sd * (S.F0 + tau * (S.a1 + tau * (S.a2 + tau * S.a3))) - f;
    if (r == 0.0) break;
    const double gp = sd * (S.a1 + tau * (2.0 * S.a2 + 3.0 * S.a3 * tau));
    if (dd * r < 0.0)
      blo = tau;
    else
      bhi = tau;
    double tn = tau - r * rcp_nr1(gp);
    if (!(tn > blo && tn < bhi)) tn = 0.5 * (blo + bhi);
    const double step = fabs(tn - tau);
    tau = tn;
    if (step <= tol || !(bhi - blo > tol)) break;
  }
  return tau;
}

// psi = 2 pi f (t_i + tau) - s Phi_V(t_i + tau): the large part
// 2 pi f t_i - s Phi_V,i in double-double, reduced modulo 2 pi, plus the
// segment-local part in double.
__device__ __forceinline__ double phase_psi(double f, double tau, double sd, double m, double n, const SegData& S) {
  const dd ft = two_prod(f, S.ti);
  dd q = two_prod(ft.hi, kTwoPiHi);
  q.lo = __builtin_fma(ft.hi, kTwoPiLo, __builtin_fma(ft.lo, kTwoPiHi, q.lo));
  const dd pm = two_prod(m, S.Ppi);
  const dd pn = two_prod(n, S.Pri);
  dd z = two_sum(pm.hi, pn.hi);
  z.lo += pm.lo + pn.lo;
  dd b = two_sum(q.hi, -sd * z.hi);
  b.lo += q.lo - sd * z.lo;
  const double kk = rint(b.hi * kInvTwoPi);
  const dd kc = two_prod(kk, kTwoPiHi);
  const double red = (b.hi - kc.hi) + ((b.lo - kc.lo) - kk * kTwoPiLo);
  const double small = tau * (kTwoPiHi * f - sd * (S.b1 + tau * (S.b2 + tau * S.b3)));
  return red + small;
}

// sin and cos of x in double precision: Cody-Waite reduction by pi/2 split
// into three parts (33 + 33 + 53 bits, each product subtracted with one
// fused multiply-add), then the Taylor series of sin and cos on
// [-pi/4, pi/4] (terms up to r^17 and r^18; the first omitted terms are
// below 1e-19) and a quadrant rotation.
__device__ __forceinline__ void sincos_cw(double x, double* sn, double* cs) {
  constexpr double kPio2A = 1.5707963267341256;
  constexpr double kPio2B = 6.077100506303966e-11;
  constexpr double kPio2C = 2.0222662487959506e-21;
  constexpr double k2OverPi = 0.6366197723675814;
  const double k = rint(x * k2OverPi);
  double r = __builtin_fma(-k, kPio2A, x);
  r = __builtin_fma(-k, kPio2B, r);
  r = __builtin_fma(-k, kPio2C, r);
  const double z = r * r;
  double ps = 2.8114572543455206e-15;
  ps = __builtin_fma(ps, z, -7.647163731819816e-13);
  ps = __builtin_fma(ps, z, 1.6059043836821613e-10);
  ps = __builtin_fma(ps, z, -2.505210838544172e-08);
  ps = __builtin_fma(ps, z, 2.7557319223985893e-06);
  ps = __builtin_fma(ps, z, -0.0001984126984126984);
  ps = __builtin_fma(ps, z, 0.008333333333333333);
  ps = __builtin_fma(ps, z, -0.16666666666666666);
  const double s_r = __builtin_fma(r * z, ps, r);
  double pc = -1.5619206968586225e-16;
  pc = __builtin_fma(pc, z, 4.779477332387385e-14);
  pc = __builtin_fma(pc, z, -1.1470745597729725e-11);
  pc = __builtin_fma(pc, z, 2.08767569878681e-09);
  pc = __builtin_fma(pc, z, -2.755731922398589e-07);
  pc = __builtin_fma(pc, z, 2.48015873015873e-05);
  pc = __builtin_fma(pc, z, -0.001388888888888889);
  pc = __builtin_fma(pc, z, 0.041666666666666664);
  pc = __builtin_fma(pc, z, -0.5);
  const double c_r = __builtin_fma(z, pc, 1.0);
  const int q = ((int)(long long)k) & 3;
  const double s1 = (q & 1) ? c_r : s_r;
  const double c1 = (q & 1) ? s_r : c_r;
  *sn = (q & 2) ? -s1 : s1;
  *cs = ((q + 1) & 2) ? -c1 : c1;
}

// E = e^{i psi} G and the amplitude spline value A at the root (FP64).
__device__ __forceinline__ void root_terms64(double f, double tau, double sd, int d, double m, double n,
                                             const SegData& S, const double* __restrict__ ac_seg, double2& E,
                                             double2& A) {
  const double gd = sd * (S.a1 + tau * (2.0 * S.a2 + 3.0 * S.a3 * tau));
  const double gdd = sd * (2.0 * S.a2 + 6.0 * S.a3 * tau);
  const double psi = phase_psi(f, tau, sd, m, n, S);
  const double2 G = spa_factor64(gd, gdd, d);
  double sn, cs;
  sincos_cw(psi, &sn, &cs);
  E = make_double2(cs * G.x - sn * G.y, cs * G.y + sn * G.x);
  const double* c = ac_seg;
  A = make_double2(c[0] + tau * (c[2] + tau * (c[4] + tau * c[6])), c[1] + tau * (c[3] + tau * (c[5] + tau * c[7])));
}

// Mixed precision: root, derivatives, phase and its reduction in FP64; the
// factor, sincos and the (normalised) amplitude spline in FP32.
__device__ __forceinline__ void root_terms32(double f, double tau, double sd, int d, double m, double n,
                                             const SegData& S, const float* __restrict__ ac32_seg, float2& E,
                                             float2& A) {
  const double gd = sd * (S.a1 + tau * (2.0 * S.a2 + 3.0 * S.a3 * tau));
  const double gdd = sd * (2.0 * S.a2 + 6.0 * S.a3 * tau);
  const double psi = phase_psi(f, tau, sd, m, n, S);
  const double psr = psi - kTwoPiHi * rint(psi * kInvTwoPi);
  const float2 G = spa_factor32(gd, gdd, d);
  float sn, cs;
  sincosf((float)psr, &sn, &cs);
  E = make_float2(cs * G.x - sn * G.y, cs * G.y + sn * G.x);
  const float u = (float)(tau / S.h);
  const float* c = ac32_seg;
  A = make_float2(c[0] + u * (c[2] + u * (c[4] + u * c[6])), c[1] + u * (c[3] + u * (c[5] + u * c[7])));
}

}  // namespace fdemri
