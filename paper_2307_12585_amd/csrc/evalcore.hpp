// Per-root arithmetic of the frequency-domain mode sum (Sec. 2.2), shared
// by the forward gather and the adjoint so that both evaluate bit-identical
// roots, phases and factors.
//
// For a voice (m, n) on a monotonic piece with sign s and direction d, and a
// bin f whose root lies in spline segment i (Eq. cubic_equation):
//   |F_V|(t_i + tau) = G0 + q1 tau + q2 tau^2 + q3 tau^3,
//   s Phi_V(t_i + tau) = s Phi_V,i + r1 tau + r2 tau^2 + r3 tau^3,
// with G0 = (s m) F_phi,i + (s n) F_r,i from the knot data and q_k, r_k the
// spline coefficients of the fundamental frequencies and phases weighted by
// s m and s n (the sign is folded into the mode numbers, which is exact).

#pragma once

#include "spa.hpp"

namespace fdemri {

struct SegData {
  double ti, h, G0, G1;   // knot time, segment length, |F_V| at both knots
  double q1, q2, q3;      // |F_V| spline coefficients
  double r1, r2, r3;      // s Phi_V spline coefficients
  double Ppi, Pri;        // Phi_phi, Phi_r at t_i reduced modulo 2 pi (reduce_2pi)
};

// x modulo 2 pi, in [-pi, pi]: the multiple k of 2 pi is removed with 2 pi
// split into hi + lo parts and k * hi formed exactly, so the result carries
// the rounding error of x only.
__device__ __forceinline__ double reduce_2pi(double x) {
  const double k = rint(x * kInvTwoPi);
  const dd kc = two_prod(k, kTwoPiHi);
  return ((x - kc.hi) - kc.lo) - k * kTwoPiLo;
}

// Bracket of the root inside segment i of piece P: [tl, th] in tau, with
// |F_V| = gl, gh at its ends (piece end values at the piece's first/last
// segment, knot values elsewhere).  A piece over the whole trajectory has
// knot values at both ends, and so does a wave none of whose lanes is in the
// first or last segment of its piece: their bracket is the segment's
// (wave-uniform tests that save the per-lane selects).
struct Bracket {
  double tl, th, gl, gh;
};

__device__ __forceinline__ Bracket make_bracket(const Piece& P, int i, const SegData& S) {
  Bracket B;
  if (P.whole || !__any(i == P.seg_a || i == P.seg_b)) {
    B = Bracket{0.0, S.h, S.G0, S.G1};
  } else {
    // an empty volatile statement keeps this a branch: if-converted, both
    // sides would be computed with per-lane selects for every piece
    asm volatile("");
    const bool first = (i == P.seg_a), last = (i == P.seg_b);
    B.tl = first ? P.tau_a : 0.0;
    B.th = last ? P.tau_b : S.h;
    B.gl = first ? P.g_a : S.G0;
    B.gh = last ? P.g_b : S.G1;
  }
  return B;
}

// Root of G0 + q1 tau + q2 tau^2 + q3 tau^3 = f on [tl, th] (|F_V|
// monotonic there with direction d).  Secant start from the bracket ends,
// then Halley steps on p(tau) = |F_V|(t_i + tau) - f.  After a Halley step
// of length x the error is about (p2^2 / (4 p1^2) - p3 / (6 p1)) x^3, with
// p1, p2, p3 the first three derivatives of p; a step is accepted as the
// root once the iterate lies where that holds (|p p2| <= p1^2 / 2) and the
// predicted error is below the tolerance.  On smooth trajectories the first
// step from the secant start is accepted; otherwise the iteration goes on
// from that step, inside the bracket narrowed by the sign of p at the start,
// with every step kept inside the shrinking bracket (bisection when a step
// leaves it).
__device__ __forceinline__ double solve_root(double f, double dd, const SegData& S, const Bracket& B) {
  double tau0 = B.tl;
  const double dg = B.gh - B.gl;
  if (dg != 0.0) tau0 = B.tl + (f - B.gl) * (B.th - B.tl) * rcp_nr1(dg);
  tau0 = fmin(fmax(tau0, B.tl), B.th);
  const double tol = 4e-16 * fmax(S.h, 1.0);
  const double c0 = S.G0 - f;
  const double q1 = S.q1, q2 = S.q2, q3 = S.q3;
  const double q2x2 = 2.0 * q2, q3x3 = 3.0 * q3, q3x6 = 6.0 * q3, aq3 = fabs(q3);
  // first Halley step, accepted when the error estimate allows
  double blo = B.tl, bhi = B.th, tau;
  {
    const double r = c0 + tau0 * (q1 + tau0 * (q2 + tau0 * q3));
    const double p1 = q1 + tau0 * (q2x2 + q3x3 * tau0);
    const double p2 = q2x2 + q3x6 * tau0;
    const double p1s = p1 * p1, rp2 = r * p2;
    const double tn = tau0 - 2.0 * r * p1 * rcp_nr1(2.0 * p1s - rp2);
    const double step = fabs(tn - tau0);
    if (r == 0.0) return tau0;
    if (tn >= B.tl && tn <= B.th &&
        (step <= tol ||
         (fabs(rp2) <= 0.5 * p1s && step * step * step * (0.25 * p2 * p2 + aq3 * fabs(p1)) <= tol * p1s)))
      return tn;
    // not accepted: the start point's sign narrows the bracket, and the
    // iteration continues from the step just taken
    if (dd * r < 0.0)
      blo = tau0;
    else
      bhi = tau0;
    tau = (tn > blo && tn < bhi) ? tn : 0.5 * (blo + bhi);
  }
  for (int it = 0; it < 100; ++it) {
    const double r = c0 + tau * (q1 + tau * (q2 + tau * q3));
    if (r == 0.0) break;
    const double p1 = q1 + tau * (q2x2 + q3x3 * tau);
    const double p2 = q2x2 + q3x6 * tau;
    if (dd * r < 0.0)
      blo = tau;
    else
      bhi = tau;
    const double p1s = p1 * p1, rp2 = r * p2;
    double tn = tau - 2.0 * r * p1 * rcp_nr1(2.0 * p1s - rp2);
    const bool inside = (tn > blo && tn < bhi);
    if (!inside) tn = 0.5 * (blo + bhi);
    const double step = fabs(tn - tau);
    tau = tn;
    if (step <= tol || !(bhi - blo > tol)) break;
    if (inside && fabs(rp2) <= 0.5 * p1s && step * step * step * (0.25 * p2 * p2 + aq3 * fabs(p1)) <= tol * p1s)
      break;
  }
  return tau;
}

// psi = 2 pi f (t_i + tau) - s Phi_V(t_i + tau) up to a multiple of 2 pi,
// with w = 2 pi f and (ms, ns) = (s m, s n).  The large part is taken modulo
// 2 pi without double-double products of the phases: f t_i is formed exactly
// as a two-product and only its fractional part is kept, and since ms and
// ns are integers, ms Phi_phi,i + ns Phi_r,i equals (mod 2 pi) the same
// combination of the knot phases reduced modulo 2 pi, at most a few hundred
// radians here.  The segment-local part is added in double.
__device__ __forceinline__ double phase_psi(double f, double w, double tau, double ms, double ns, const SegData& S) {
  const dd ft = two_prod(f, S.ti);
  const double fr = (ft.hi - rint(ft.hi)) + ft.lo;
  const double big = kTwoPiHi * fr - __builtin_fma(ms, S.Ppi, ns * S.Pri);
  const double small = tau * (w - (S.r1 + tau * (S.r2 + tau * S.r3)));
  return big + small;
}

// sin and cos of x in double precision: Cody-Waite reduction by pi split
// into two parts (a 34-bit head, so k times it is exact for the multiples
// that occur, and the rounded remainder), each product subtracted with one
// fused multiply-add; then on r in [-pi/2, pi/2]
//   sin r = r + r z P(z),  cos r = 1 - z/2 + z^2 Q(z),  z = r^2,
// with P, Q degree-7 least-squares fits in extended precision
// (gen_sincos_coeffs.py; approximation errors 1.3e-18 relative and 1.0e-19),
// and the sign (-1)^k of the multiple k of pi given to both results (one
// exclusive or of the sign bit each: no quadrant selects).  The phases
// passed here are reduced modulo 2 pi up to a few hundred radians and the
// segment-local part, a few thousand radians at most, so k fits an int.
__device__ __forceinline__ void sincos_cw(double x, double* sn, double* cs) {
  constexpr double kPiA = 3.1415926534682512;
  constexpr double kPiB = 1.2154201013012384e-10;
  constexpr double kInvPi = 0.3183098861837907;
  const double k = rint(x * kInvPi);
  double r = __builtin_fma(-k, kPiA, x);
  r = __builtin_fma(-k, kPiB, r);
  const double z = r * r;
  double ps = __builtin_fma(2.7314520351307035e-15, z, -7.643970924523278e-13);
  ps = fma_sc(ps, z, 1.605897733376295e-10);
  ps = fma_sc(ps, z, -2.5052107617354543e-08);
  ps = fma_sc(ps, z, 2.755731921916633e-06);
  ps = fma_sc(ps, z, -0.00019841269841254988);
  ps = fma_sc(ps, z, 0.008333333333333316);
  ps = fma_sc(ps, z, -0.16666666666666666);
  const double s_r = __builtin_fma(r * z, ps, r);
  double pc = __builtin_fma(-1.5218671473552762e-16, z, 4.7778782111543295e-14);
  pc = fma_sc(pc, z, -1.1470712282450332e-11);
  pc = fma_sc(pc, z, 2.087675660303868e-09);
  pc = fma_sc(pc, z, -2.755731922157097e-07);
  pc = fma_sc(pc, z, 2.4801587301579858e-05);
  pc = fma_sc(pc, z, -0.001388888888888888);
  pc = fma_sc(pc, z, 0.041666666666666664);
  const double c_r = __builtin_fma(z * z, pc, __builtin_fma(-0.5, z, 1.0));
  const long long sign = (long long)((uint32_t)cvt_i32_sat(k) << 31) << 32;
  *sn = __longlong_as_double(__double_as_longlong(s_r) ^ sign);
  *cs = __longlong_as_double(__double_as_longlong(c_r) ^ sign);
}

// sin and cos of psi for the mixed path: the reduction by pi/2 in FP64 (the
// two-part split of sincos_cw), then degree-2 least-squares polynomials in
// FP32 on [-pi/4, pi/4] (gen_sincos_coeffs.py; approximation errors 1.4e-8
// relative for sin and 7.6e-10 for cos, below FP32 rounding) and the
// quadrant rotation.
__device__ __forceinline__ void sincos_mixed(double x, float* sn, float* cs) {
  constexpr double kPio2A = 1.5707963267341256;
  constexpr double kPio2B = 6.077100506506192e-11;
  constexpr double k2OverPi = 0.6366197723675814;
  const double k = rint(x * k2OverPi);
  double r = __builtin_fma(-k, kPio2A, x);
  r = __builtin_fma(-k, kPio2B, r);
  const float rf = (float)r;
  const float z = rf * rf;
  float ps = __builtin_fmaf(-0.00019587949872019718f, z, 0.008332748634609668f);
  ps = __builtin_fmaf(ps, z, -0.16666664665122977f);
  const float s_r = __builtin_fmaf(rf * z, ps, rf);
  float pc = __builtin_fmaf(2.4547991314265332e-05f, z, -0.001388830333962966f);
  pc = __builtin_fmaf(pc, z, 0.04166666466184568f);
  const float c_r = __builtin_fmaf(z * z, pc, __builtin_fmaf(-0.5f, z, 1.0f));
  const int q = cvt_i32_sat(k) & 3;
  const float s1 = (q & 1) ? c_r : s_r;
  const float c1 = (q & 1) ? s_r : c_r;
  *sn = (q & 2) ? -s1 : s1;
  *cs = ((q + 1) & 2) ? -c1 : c1;
}

// E = e^{i psi} G and the amplitude spline value A at the root; w = 2 pi f,
// (ms, ns) = (s m, s n).
// The amplitude spline coefficients of one segment, (re, im) pairs in
// ascending powers: read as a whole by the caller, so that the loads can be
// issued as soon as the segment is known and their latency overlaps the root
// solve.
struct AmpSeg64 {
  double2 c[4];
};
struct AmpSeg32 {
  float4 lo, hi;  // (re0, im0, re1, im1), (re2, im2, re3, im3)
};

__device__ __forceinline__ AmpSeg64 load_amp64(const double* __restrict__ ac_seg) {
  const double2* q = (const double2*)ac_seg;
  return AmpSeg64{{q[0], q[1], q[2], q[3]}};
}

__device__ __forceinline__ AmpSeg32 load_amp32(const float* __restrict__ ac32_seg) {
  const float4* q = (const float4*)ac32_seg;
  return AmpSeg32{q[0], q[1]};
}

// E = e^{i psi} G at the root (FP64).
__device__ __forceinline__ double2 root_E64(double f, double w, double tau, int d, double ms, double ns,
                                            const SegData& S) {
  const double gd = S.q1 + tau * (2.0 * S.q2 + 3.0 * S.q3 * tau);
  const double gdd = 2.0 * S.q2 + 6.0 * S.q3 * tau;
  const double psi = phase_psi(f, w, tau, ms, ns, S);
  const double2 G = spa_factor64(gd, gdd, d);
  double sn, cs;
  sincos_cw(psi, &sn, &cs);
  return make_double2(cs * G.x - sn * G.y, cs * G.y + sn * G.x);
}

// The amplitude spline of one segment at tau (FP64).
__device__ __forceinline__ double2 amp64(const AmpSeg64& c, double tau) {
  return make_double2(c.c[0].x + tau * (c.c[1].x + tau * (c.c[2].x + tau * c.c[3].x)),
                      c.c[0].y + tau * (c.c[1].y + tau * (c.c[2].y + tau * c.c[3].y)));
}

__device__ __forceinline__ void root_terms64(double f, double w, double tau, int d, double ms, double ns,
                                             const SegData& S, const AmpSeg64& c, double2& E, double2& A) {
  E = root_E64(f, w, tau, d, ms, ns, S);
  A = amp64(c, tau);
}

__device__ __forceinline__ void root_terms64(double f, double w, double tau, int d, double ms, double ns,
                                             const SegData& S, const double* __restrict__ ac_seg, double2& E,
                                             double2& A) {
  root_terms64(f, w, tau, d, ms, ns, S, load_amp64(ac_seg), E, A);
}

// Mixed precision: root, derivatives, phase and its reduction in FP64; the
// factor, sincos and the (normalised) amplitude spline in FP32.
__device__ __forceinline__ float2 root_E32(double f, double w, double tau, int d, double ms, double ns,
                                           const SegData& S) {
  const double gd = S.q1 + tau * (2.0 * S.q2 + 3.0 * S.q3 * tau);
  const double gdd = 2.0 * S.q2 + 6.0 * S.q3 * tau;
  const double psi = phase_psi(f, w, tau, ms, ns, S);
  const float2 G = spa_factor32(gd, gdd, d);
  float sn, cs;
  sincos_mixed(psi, &sn, &cs);
  return make_float2(cs * G.x - sn * G.y, cs * G.y + sn * G.x);
}

// tau / h to FP32 accuracy: the variable of the normalised FP32 amplitude.
__device__ __forceinline__ float amp_u32(double tau, const SegData& S) {
  return (float)tau * __builtin_amdgcn_rcpf((float)S.h);
}

__device__ __forceinline__ float2 amp32(const AmpSeg32& c, float u) {
  return make_float2(c.lo.x + u * (c.lo.z + u * (c.hi.x + u * c.hi.z)), c.lo.y + u * (c.lo.w + u * (c.hi.y + u * c.hi.w)));
}

__device__ __forceinline__ void root_terms32(double f, double w, double tau, int d, double ms, double ns,
                                             const SegData& S, const AmpSeg32& c, float2& E, float2& A) {
  E = root_E32(f, w, tau, d, ms, ns, S);
  A = amp32(c, amp_u32(tau, S));
}

__device__ __forceinline__ void root_terms32(double f, double w, double tau, int d, double ms, double ns,
                                             const SegData& S, const float* __restrict__ ac32_seg, float2& E,
                                             float2& A) {
  root_terms32(f, w, tau, d, ms, ns, S, load_amp32(ac32_seg), E, A);
}

}  // namespace fdemri
