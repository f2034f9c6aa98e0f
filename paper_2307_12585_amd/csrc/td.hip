// Time-domain voice sum (Eq. wave_voice, polarizations of Eq. main_wave) on
// a uniform time grid, from the same splines and mode factors as the
// frequency-domain path: the comparison model of the paper's FD/TD timing
// study (Sec. 3.2), whose transform is compared with the FD sum.
//
// For a mode row with amplitude A(t), phase Phi(t) = m Phi_phi(t) + n Phi_r(t)
// and fused polarization factors c_+, c_x (partner (l,-m,-n) included, as in
// the FD gather), h = h_+ - i h_x summed over the row's voices gives
//   h_+(t) = 2 Re(X c_+),   h_x(t) = 2 Re(X c_x),   X = A(t) e^{-i Phi(t)}.
// Per sample the knot phases (reduced modulo 2 pi) plus the segment-local
// cubic give Phi_phi and Phi_r reduced modulo 2 pi once; per row
// m Phi_phi + n Phi_r is then a few hundred radians at most, and sin, cos
// come from the same kernel as the FD path.  One thread per sample, rows in
// table order; samples outside [t_0, t_{K-1}] are 0.
#include "evalcore.hpp"

namespace fdemri {

constexpr int kTdThreads = 256;

// t_k = t0 + k dt with the product rounded before the sum (no fused
// multiply-add), the way the grid is usually formed on the host.
__device__ __forceinline__ double sample_time(double t0, double dt, int k) {
#pragma clang fp contract(off)
  const double kd = (double)k * dt;
  return t0 + kd;
}

struct TdArgs {
  int K, Nm, Nt;
  double t0, dt;
  const double* t;       // [K] knot times
  const double* Phiphi;  // [K]
  const double* Phir;    // [K]
  const double* tcoef;   // [4][K-1][4]
  const double* acoef;   // [Nm][K-1][8]
  const ModeConst* modes;
  double* hp;  // [Nt]
  double* hc;  // [Nt]
};

__global__ __launch_bounds__(kTdThreads) void td_kernel(TdArgs a) {
  // knot times in LDS for the segment search
  __shared__ double s_t[kMaxKnots];
  const int K = a.K, nseg = K - 1;
  for (int i = threadIdx.x; i < K; i += kTdThreads) s_t[i] = a.t[i];
  __syncthreads();
  const int k = (int)blockIdx.x * kTdThreads + (int)threadIdx.x;
  const double ts = sample_time(a.t0, a.dt, k);
  const bool in = k < a.Nt && ts >= s_t[0] && ts <= s_t[K - 1];
  // segment: largest i in [0, K-2] with t_i <= ts (binary search)
  int lo = 0, hi = nseg - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (s_t[mid] <= ts)
      lo = mid;
    else
      hi = mid - 1;
  }
  const int seg = lo;
  const double tau = in ? ts - s_t[seg] : 0.0;
  // Phi_phi, Phi_r at the sample, reduced modulo 2 pi: knot value reduced
  // first, then the local cubic added and the sum reduced again
  const double* cP = a.tcoef + ((size_t)2 * nseg + seg) * 4;
  const double* cR = a.tcoef + ((size_t)3 * nseg + seg) * 4;
  const double pp = reduce_2pi(reduce_2pi(a.Phiphi[seg]) + tau * (cP[1] + tau * (cP[2] + tau * cP[3])));
  const double pr = reduce_2pi(reduce_2pi(a.Phir[seg]) + tau * (cR[1] + tau * (cR[2] + tau * cR[3])));
  double hp = 0.0, hc = 0.0;
  if (in) {
    const double* ac = a.acoef + (size_t)seg * 8;
    const kconst ModeConst* md = (const kconst ModeConst*)a.modes;
    for (int mu = 0; mu < a.Nm; ++mu) {
      const ModeConst c = md[mu];
      const double* q = ac + (size_t)mu * nseg * 8;
      const double Ar = q[0] + tau * (q[2] + tau * (q[4] + tau * q[6]));
      const double Ai = q[1] + tau * (q[3] + tau * (q[5] + tau * q[7]));
      double sn, cs;
      sincos_cw(__builtin_fma(c.m, pp, c.n * pr), &sn, &cs);
      // X = A e^{-i psi}
      const double Xr = Ar * cs + Ai * sn, Xi = Ai * cs - Ar * sn;
      hp += Xr * c.cp_re - Xi * c.cp_im;
      hc += Xr * c.cx_re - Xi * c.cx_im;
    }
  }
  if (k < a.Nt) {
    a.hp[k] = 2.0 * hp;
    a.hc[k] = 2.0 * hc;
  }
}

hipError_t launch_td(int K, int Nm, const double* t, const double* Phiphi, const double* Phir, const double* tcoef,
                     const double* acoef, const ModeConst* modes, double t0, double dt, int Nt, double* hp, double* hc,
                     hipStream_t stream) {
  if (Nt <= 0) return hipSuccess;
  TdArgs a;
  a.K = K;
  a.Nm = Nm;
  a.Nt = Nt;
  a.t0 = t0;
  a.dt = dt;
  a.t = t;
  a.Phiphi = Phiphi;
  a.Phir = Phir;
  a.tcoef = tcoef;
  a.acoef = acoef;
  a.modes = modes;
  a.hp = hp;
  a.hc = hc;
  td_kernel<<<(Nt + kTdThreads - 1) / kTdThreads, kTdThreads, 0, stream>>>(a);
  return hipGetLastError();
}

}  // namespace fdemri
