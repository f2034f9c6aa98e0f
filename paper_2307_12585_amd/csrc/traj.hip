// The sparse inspiral trajectory on the device (Sec. 2.1: the adiabatic
// orbit is integrated to ~100 points before the mode sum; here the toy
// orbit-averaged fluxes of the synthetic workloads), one thread per
// waveform of a batch:
//   dp/dt = -(64/5) q (1-e^2)^{3/2} p^{-3} (1 + 7e^2/8) / M_s,
//   de/dt = -(304/15) q e (1-e^2)^{3/2} p^{-4} (1 + 121e^2/304) / M_s,
//   dPhi_phi/dt = Omega_phi / M_s,  dPhi_r/dt = Omega_r / M_s,
//   Omega_phi = p^{-3/2} (1-e^2)^{3/2},  Omega_r = Omega_phi sqrt(1 - 6/p),
// with q = mu/M and M_s = M G M_sun/c^3, from t = 0 to T or to the plunge
// p = 6 + 2e + 0.1, whichever comes first; K knots uniform in [0, t_end].
//
// Integrator: the Dormand-Prince 5(4) embedded pair with the usual error
// control (scaled RMS of the 4th/5th-order difference, step factor
// 0.9 err^{-1/5} within [0.2, 5]).  Pass 1 finds t_end (the plunge located
// by secant iterations on the length of the last step, each trial a full
// step from the last accepted state); pass 2 integrates again with steps
// clipped to land on every knot time.  Every thread leaves its loops after at
// most kMaxSteps steps per pass (a flag is raised if that bound is hit).
#include "fdemri_internal.hpp"

namespace fdemri {

constexpr double kMtsun = 4.925490947641267e-6;  // G M_sun / c^3 in s
constexpr int kMaxSteps = 2000000;

struct TrajIn {
  double M, mu, p0, e0, T, Phiphi0, Phir0;
};

struct Rhs {
  double q, Ms;
  __device__ void operator()(const double y[4], double d[4]) const {
    const double p = y[0], e = y[1];
    const double e2 = e * e, one_e2 = 1.0 - e2;
    const double s = one_e2 * sqrt(one_e2);  // (1 - e^2)^{3/2}
    const double ip = 1.0 / p;
    const double ip3 = ip * ip * ip;
    d[0] = -(64.0 / 5.0) * q * s * ip3 * (1.0 + 0.875 * e2) / Ms;
    d[1] = -(304.0 / 15.0) * q * e * s * ip3 * ip * (1.0 + (121.0 / 304.0) * e2) / Ms;
    const double om_phi = ip * sqrt(ip) * s;
    d[2] = om_phi / Ms;
    d[3] = om_phi * sqrt(1.0 - 6.0 * ip) / Ms;
  }
};

// One Dormand-Prince step of length h from (y, k1 = f(y)): the 5th-order
// solution in yn, f(yn) in k7 (first stage of the next step) and the
// scaled error norm.
__device__ __forceinline__ double dp45_step(const Rhs& f, const double y[4], const double k1[4], double h,
                                            double yn[4], double k7[4]) {
  constexpr double a21 = 1.0 / 5.0;
  constexpr double a31 = 3.0 / 40.0, a32 = 9.0 / 40.0;
  constexpr double a41 = 44.0 / 45.0, a42 = -56.0 / 15.0, a43 = 32.0 / 9.0;
  constexpr double a51 = 19372.0 / 6561.0, a52 = -25360.0 / 2187.0, a53 = 64448.0 / 6561.0, a54 = -212.0 / 729.0;
  constexpr double a61 = 9017.0 / 3168.0, a62 = -355.0 / 33.0, a63 = 46732.0 / 5247.0, a64 = 49.0 / 176.0,
                   a65 = -5103.0 / 18656.0;
  constexpr double b1 = 35.0 / 384.0, b3 = 500.0 / 1113.0, b4 = 125.0 / 192.0, b5 = -2187.0 / 6784.0,
                   b6 = 11.0 / 84.0;
  // b - b* (5th minus embedded 4th order weights)
  constexpr double e1 = 71.0 / 57600.0, e3 = -71.0 / 16695.0, e4 = 71.0 / 1920.0, e5 = -17253.0 / 339200.0,
                   e6 = 22.0 / 525.0, e7 = -1.0 / 40.0;
  constexpr double atol[4] = {1e-12, 1e-14, 1e-9, 1e-9};
  constexpr double rtol = 1e-12;
  double k2[4], k3[4], k4[4], k5[4], k6[4], z[4];
  for (int i = 0; i < 4; ++i) z[i] = y[i] + h * a21 * k1[i];
  f(z, k2);
  for (int i = 0; i < 4; ++i) z[i] = y[i] + h * (a31 * k1[i] + a32 * k2[i]);
  f(z, k3);
  for (int i = 0; i < 4; ++i) z[i] = y[i] + h * (a41 * k1[i] + a42 * k2[i] + a43 * k3[i]);
  f(z, k4);
  for (int i = 0; i < 4; ++i) z[i] = y[i] + h * (a51 * k1[i] + a52 * k2[i] + a53 * k3[i] + a54 * k4[i]);
  f(z, k5);
  for (int i = 0; i < 4; ++i) z[i] = y[i] + h * (a61 * k1[i] + a62 * k2[i] + a63 * k3[i] + a64 * k4[i] + a65 * k5[i]);
  f(z, k6);
  for (int i = 0; i < 4; ++i) yn[i] = y[i] + h * (b1 * k1[i] + b3 * k3[i] + b4 * k4[i] + b5 * k5[i] + b6 * k6[i]);
  f(yn, k7);
  double err = 0.0;
  for (int i = 0; i < 4; ++i) {
    const double ei = h * (e1 * k1[i] + e3 * k3[i] + e4 * k4[i] + e5 * k5[i] + e6 * k6[i] + e7 * k7[i]);
    const double sc = atol[i] + rtol * fmax(fabs(y[i]), fabs(yn[i]));
    err += (ei / sc) * (ei / sc);
  }
  return sqrt(0.25 * err);
}

__device__ __forceinline__ double plunge_gap(const double y[4]) { return y[0] - (6.0 + 2.0 * y[1] + 0.1); }

// Step-size factor after a step with error norm err (0.2 for a rejected
// non-finite trial).
__device__ __forceinline__ double step_factor(double err) {
  if (!(err == err)) return 0.2;
  return err == 0.0 ? 5.0 : fmin(5.0, fmax(0.2, 0.9 * pow(err, -0.2)));
}

// out: [B][7][K] (t, F_phi, F_r, Phi_phi, Phi_r, p, e).
__global__ __launch_bounds__(64) void traj_kernel(const TrajIn* __restrict__ in, int B, int K, double* __restrict__ out,
                                                  uint32_t* __restrict__ flag_word) {
  const int b = (int)blockIdx.x * 64 + (int)threadIdx.x;
  if (b >= B) return;
  const TrajIn P = in[b];
  const Rhs f{P.mu / P.M, P.M * kMtsun};
  const double y0[4] = {P.p0, P.e0, P.Phiphi0, P.Phir0};
  bool capped = false;

  // pass 1: t_end.  First step: a small fraction of the radiation-reaction
  // time p / |dp/dt| (the controller grows it).
  double t = 0.0, y[4], k1[4], yn[4], k7[4];
  for (int i = 0; i < 4; ++i) y[i] = y0[i];
  f(y, k1);
  const double h0 = fmin(P.T, 1e-4 * P.p0 / fabs(k1[0]));
  double h = h0;
  double t_end = P.T;
  for (int it = 0;; ++it) {
    if (it >= kMaxSteps) {
      capped = true;
      t_end = t;
      break;
    }
    const double hs = fmin(h, P.T - t);
    const double err = dp45_step(f, y, k1, hs, yn, k7);
    if (!(err <= 1.0)) {  // rejected (also when the trial left the domain: NaN)
      h = hs * step_factor(err);
      continue;
    }
    if (plunge_gap(yn) <= 0.0) {
      // the plunge lies in (t, t + hs]: secant iterations on the step length
      double ha = 0.0, ga = plunge_gap(y), hb = hs, gb = plunge_gap(yn);
      double hc = hs;
      for (int j = 0; j < 60; ++j) {
        hc = ha + (hb - ha) * ga / (ga - gb);
        if (!(hc > ha && hc < hb)) hc = 0.5 * (ha + hb);
        double ytmp[4], ktmp[4];
        dp45_step(f, y, k1, hc, ytmp, ktmp);
        const double gc = plunge_gap(ytmp);
        if (gc > 0.0) {
          ha = hc;
          ga = gc;
        } else {
          hb = hc;
          gb = gc;
        }
        if (fabs(gc) <= 1e-14 * y[0] || hb - ha <= 1e-15 * (t + hb)) break;
      }
      t_end = t + hc;
      break;
    }
    const bool last = (hs == P.T - t);
    t = last ? P.T : t + hs;
    for (int i = 0; i < 4; ++i) {
      y[i] = yn[i];
      k1[i] = k7[i];
    }
    if (last) {
      t_end = P.T;
      break;
    }
    h = hs * step_factor(err);
  }

  // pass 2: the knots
  double* o = out + (size_t)b * 7 * K;
  const double Ms = f.Ms, two_pi_Ms = 2.0 * kPi * Ms;
  auto emit = [&](int j, double tj, const double* yy) {
    const double p = yy[0], e = yy[1];
    const double one_e2 = 1.0 - e * e;
    const double om_phi = pow(p, -1.5) * one_e2 * sqrt(one_e2);
    const double om_r = om_phi * sqrt(1.0 - 6.0 / p);
    o[0 * K + j] = tj;
    o[1 * K + j] = om_phi / two_pi_Ms;
    o[2 * K + j] = om_r / two_pi_Ms;
    o[3 * K + j] = yy[2];
    o[4 * K + j] = yy[3];
    o[5 * K + j] = p;
    o[6 * K + j] = e;
  };
  t = 0.0;
  for (int i = 0; i < 4; ++i) y[i] = y0[i];
  f(y, k1);
  emit(0, 0.0, y);
  h = fmin(t_end, h0);
  int j = 1;
  const double dtk = t_end / (double)(K - 1);
  int steps = 0;
  while (j < K) {
    if (++steps > kMaxSteps) {
      capped = true;
      for (; j < K; ++j) emit(j, j == K - 1 ? t_end : (double)j * dtk, y);
      break;
    }
    const double tk = (j == K - 1) ? t_end : (double)j * dtk;
    const double hs = fmin(h, tk - t);
    if (!(hs > 0.0)) {
      emit(j, tk, y);
      ++j;
      continue;
    }
    const double err = dp45_step(f, y, k1, hs, yn, k7);
    if (!(err <= 1.0)) {
      h = hs * step_factor(err);
      continue;
    }
    const bool land = (hs == tk - t);
    t = land ? tk : t + hs;
    for (int i = 0; i < 4; ++i) {
      y[i] = yn[i];
      k1[i] = k7[i];
    }
    if (land) {
      emit(j, tk, y);
      ++j;
    }
    // a step clipped to land on a knot does not shrink the proposal
    h = land ? fmax(h, hs * step_factor(err)) : hs * step_factor(err);
  }
  if (capped) atomicOr(flag_word, (uint32_t)FDEMRI_FLAG_TRAJ_STEPS);
}

hipError_t launch_trajectory(const void* params, int B, int K, double* out, uint32_t* flag_word, hipStream_t stream) {
  if (B <= 0) return hipSuccess;
  traj_kernel<<<(B + 63) / 64, 64, 0, stream>>>((const TrajIn*)params, B, K, out, flag_word);
  return hipGetLastError();
}

}  // namespace fdemri
