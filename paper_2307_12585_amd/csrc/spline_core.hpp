// Not-a-knot cubic spline coefficients of the trajectory and amplitude
// series (Sec. 2.1: amplitudes and phases are interpolated with not-a-knot
// cubic splines; Sec. 2.2: so are the fundamental frequencies, and their
// coefficients are fixed before the summation).
//
// The unknowns are the knot slopes s_i.  With h_i = t_{i+1} - t_i and
// delta_i = (y_{i+1} - y_i)/h_i, interior rows are
//   h_i s_{i-1} + 2(h_{i-1}+h_i) s_i + h_{i-1} s_{i+1} = 3(h_i delta_{i-1} + h_{i-1} delta_i),
// and the not-a-knot conditions (third derivative continuous at t_1 and
// t_{K-2}), with s_2 / s_{K-3} eliminated through the neighbouring interior
// row, give the two-term boundary rows
//   h_1 s_0 + (h_0+h_1) s_1 = [(2h_1^2 + 3h_0 h_1) delta_0 + h_0^2 delta_1] / (h_0+h_1),
//   (h_{n-2}+h_{n-1}) s_{n-1} + h_{n-2} s_n
//        = [h_{n-1}^2 delta_{n-2} + (2h_{n-2}^2 + 3h_{n-2}h_{n-1}) delta_{n-1}] / (h_{n-2}+h_{n-1}).
// All series of a waveform share the knots, hence the matrix.  The system is
// solved by parallel cyclic reduction with one thread per knot; a workgroup
// reduces the matrix once and carries kSeriesPerBlock right-hand sides
// through the same log2(NT) steps, so that the reduction, the barriers and
// the LDS round trips are shared by several series.  Each segment then gets
// the Hermite coefficients
//   c0 = y_i, c1 = s_i, c2 = (3 delta_i - 2 s_i - s_{i+1})/h_i,
//   c3 = (s_i + s_{i+1} - 2 delta_i)/h_i^2.
//
// Device part shared by the spline kernels and the set-up kernel that
// computes the amplitude splines beside the piece tables.
#pragma once

#include "fdemri_internal.hpp"

namespace fdemri {

constexpr int kSeriesPerBlock = 2;

template <int NT>
struct SplineLds {
  double sa[NT], sb[NT], sc[NT], sh[NT];
  double r[kSeriesPerBlock][2][NT];  // right-hand sides (re, im), then slopes
};

// log2 of the (power-of-two) thread count NT: the number of reduction steps.
template <int NT>
constexpr int pcr_steps() {
  return NT <= 1 ? 0 : 1 + pcr_steps<NT / 2>();
}

// Doubles of the table of reduction factors of one knot matrix: per step the
// factors k1, k2 of every row, then the reciprocal of every row's final
// diagonal, [2 pcr_steps + 1][NT].
template <int NT>
constexpr int pcr_factor_doubles() {
  return (2 * pcr_steps<NT>() + 1) * NT;
}

// Value of knot j of series `series` of one waveform (0..3: F_phi, F_r,
// Phi_phi, Phi_r, real; 4 + mu: the complex amplitude of mode mu).
__device__ __forceinline__ double2 series_value(int series, int j, int K, const double* __restrict__ y0,
                                                const double* __restrict__ y1, const double* __restrict__ y2,
                                                const double* __restrict__ y3, const double* __restrict__ A) {
  if (series < 4) {
    const double* y = series == 0 ? y0 : series == 1 ? y1 : series == 2 ? y2 : y3;
    return make_double2(y[j], 0.0);
  }
  return ((const double2*)A)[(size_t)(series - 4) * K + j];
}

// Row i of the knot system: matrix entries a, b, c and the right-hand sides
// of the block's series, from the knot data parked in S.r and the segment
// lengths in S.sh.  Rows past the last knot are identity rows.
template <int NT>
__device__ __forceinline__ void spline_row(const SplineLds<NT>& S, int i, int K, double& a, double& b, double& c,
                                           double rr[kSeriesPerBlock], double ri[kSeriesPerBlock]) {
  constexpr int SB = kSeriesPerBlock;
  const int n = K - 1;
  a = 0.0;
  b = 1.0;
  c = 0.0;
#pragma unroll
  for (int q = 0; q < SB; ++q) rr[q] = ri[q] = 0.0;
  if (i >= K) return;
  auto delta = [&](int q, int j, double& dr, double& di) {
    dr = (S.r[q][0][j + 1] - S.r[q][0][j]) / S.sh[j];
    di = (S.r[q][1][j + 1] - S.r[q][1][j]) / S.sh[j];
  };
  if (i == 0) {
    const double h0 = S.sh[0], h1 = S.sh[1], w = 1.0 / (h0 + h1);
    b = h1;
    c = h0 + h1;
#pragma unroll
    for (int q = 0; q < SB; ++q) {
      double d0r, d0i, d1r, d1i;
      delta(q, 0, d0r, d0i);
      delta(q, 1, d1r, d1i);
      rr[q] = ((2.0 * h1 * h1 + 3.0 * h0 * h1) * d0r + h0 * h0 * d1r) * w;
      ri[q] = ((2.0 * h1 * h1 + 3.0 * h0 * h1) * d0i + h0 * h0 * d1i) * w;
    }
  } else if (i == n) {
    const double hm = S.sh[n - 2], hl = S.sh[n - 1], w = 1.0 / (hm + hl);
    a = hm + hl;
    b = hm;
#pragma unroll
    for (int q = 0; q < SB; ++q) {
      double dmr, dmi, dlr, dli;
      delta(q, n - 2, dmr, dmi);
      delta(q, n - 1, dlr, dli);
      rr[q] = (hl * hl * dmr + (2.0 * hm * hm + 3.0 * hm * hl) * dlr) * w;
      ri[q] = (hl * hl * dmi + (2.0 * hm * hm + 3.0 * hm * hl) * dli) * w;
    }
  } else {
    const double hp = S.sh[i - 1], hi = S.sh[i];
    a = hi;
    b = 2.0 * (hp + hi);
    c = hp;
#pragma unroll
    for (int q = 0; q < SB; ++q) {
      double dpr, dpi, dir_, dii;
      delta(q, i - 1, dpr, dpi);
      delta(q, i, dir_, dii);
      rr[q] = 3.0 * (hi * dpr + hp * dir_);
      ri[q] = 3.0 * (hi * dpi + hp * dii);
    }
  }
}

// One reduction update of a right-hand side, with the fused multiply-adds
// written out so that every kernel forms it identically.
__device__ __forceinline__ double pcr_rhs(double r, double rm, double k1, double rp, double k2) {
  return __builtin_fma(-rp, k2, __builtin_fma(-rm, k1, r));
}

// Series [s0, s0 + kSeriesPerBlock) of one waveform (0..3: F_phi, F_r,
// Phi_phi, Phi_r, real; 4 + mu: the complex amplitude of mode mu), n_series
// in all, by the NT threads of the calling workgroup.
// With acoef32 (the mixed path), the amplitude series also get FP32
// coefficients in the normalised variable u = tau / h ([Nm][K-1][8]).
// FAC_IN = false: the matrix is reduced beside the right-hand sides; when
// fac is not null, the reduction factors are written to it
// ([pcr_factor_doubles<NT>()]).  FAC_IN = true: the factors are read from
// fac (written by a reduction of the same knots with the same NT) and only
// the right-hand sides are reduced: the same values without the matrix's
// divisions and LDS traffic.
template <int NT, bool FAC_IN = false>
__device__ void spline_block(SplineLds<NT>& S, int s0, int n_series, int K, const double* __restrict__ t,
                             const double* __restrict__ y0, const double* __restrict__ y1,
                             const double* __restrict__ y2, const double* __restrict__ y3,
                             const double* __restrict__ A, double* __restrict__ tcoef, double* __restrict__ acoef,
                             double* fac = nullptr, float* __restrict__ acoef32 = nullptr) {
  constexpr int SB = kSeriesPerBlock;
  constexpr int LOG = pcr_steps<NT>();
  const int i = threadIdx.x;
  const int n = K - 1;  // segments
  if (K > NT) return;   // the host never launches this; keeps every index below in bounds
  const int ns = min(SB, n_series - s0);
  // with a factor table, its entries for this row are requested first
  double kf[FAC_IN ? 2 * LOG + 1 : 1];
  if constexpr (FAC_IN) {
#pragma unroll
    for (int q = 0; q < 2 * LOG + 1; ++q) kf[q] = fac[q * NT + i];
  }
  if (i < n) S.sh[i] = t[i + 1] - t[i];
  // the data of the block's series, one knot per thread, parked in r
#pragma unroll
  for (int q = 0; q < SB; ++q) {
    const double2 y = (q < ns && i < K) ? series_value(s0 + q, i, K, y0, y1, y2, y3, A) : make_double2(0.0, 0.0);
    S.r[q][0][i] = y.x;
    S.r[q][1][i] = y.y;
  }
  __syncthreads();

  // assemble row i: matrix and right-hand sides
  double a, b, c;
  double rr[SB], ri[SB];
  spline_row<NT>(S, i, K, a, b, c, rr, ri);
  __syncthreads();  // the data in r has been read
  if constexpr (!FAC_IN) {
    S.sa[i] = a;
    S.sb[i] = b;
    S.sc[i] = c;
  }
#pragma unroll
  for (int q = 0; q < SB; ++q) {
    S.r[q][0][i] = rr[q];
    S.r[q][1][i] = ri[q];
  }
  __syncthreads();

  // parallel cyclic reduction: after the step of stride s every row couples
  // only to rows +-2s; the factors k1, k2 come from the shared matrix
  double ib;
  if constexpr (FAC_IN) {
#pragma unroll
    for (int stp = 0; stp < LOG; ++stp) {
      const int st = 1 << stp;
      const int im = i - st, ip = i + st;
      const double k1 = kf[2 * stp], k2 = kf[2 * stp + 1];
#pragma unroll
      for (int q = 0; q < SB; ++q) {
        const double rmr = (im >= 0) ? S.r[q][0][im] : 0.0, rmi = (im >= 0) ? S.r[q][1][im] : 0.0;
        const double rpr = (ip < NT) ? S.r[q][0][ip] : 0.0, rpi = (ip < NT) ? S.r[q][1][ip] : 0.0;
        rr[q] = pcr_rhs(rr[q], rmr, k1, rpr, k2);
        ri[q] = pcr_rhs(ri[q], rmi, k1, rpi, k2);
      }
      __syncthreads();
#pragma unroll
      for (int q = 0; q < SB; ++q) {
        S.r[q][0][i] = rr[q];
        S.r[q][1][i] = ri[q];
      }
      __syncthreads();
    }
    ib = kf[2 * LOG];
  } else {
    int stp = 0;
#pragma unroll 1
    for (int st = 1; st < NT; st <<= 1, ++stp) {
      const int im = i - st, ip = i + st;
      double am = 0.0, bm = 1.0, cm = 0.0, ap = 0.0, bp = 1.0, cp = 0.0;
      if (im >= 0) {
        am = S.sa[im];
        bm = S.sb[im];
        cm = S.sc[im];
      }
      if (ip < NT) {
        ap = S.sa[ip];
        bp = S.sb[ip];
        cp = S.sc[ip];
      }
      const double k1 = a / bm, k2 = c / bp;
      if (fac) {
        fac[(2 * stp) * NT + i] = k1;
        fac[(2 * stp + 1) * NT + i] = k2;
      }
#pragma unroll
      for (int q = 0; q < SB; ++q) {
        const double rmr = (im >= 0) ? S.r[q][0][im] : 0.0, rmi = (im >= 0) ? S.r[q][1][im] : 0.0;
        const double rpr = (ip < NT) ? S.r[q][0][ip] : 0.0, rpi = (ip < NT) ? S.r[q][1][ip] : 0.0;
        rr[q] = pcr_rhs(rr[q], rmr, k1, rpr, k2);
        ri[q] = pcr_rhs(ri[q], rmi, k1, rpi, k2);
      }
      const double na = -am * k1, nc = -cp * k2, nb = b - cm * k1 - ap * k2;
      __syncthreads();
      a = na;
      b = nb;
      c = nc;
      S.sa[i] = a;
      S.sb[i] = b;
      S.sc[i] = c;
#pragma unroll
      for (int q = 0; q < SB; ++q) {
        S.r[q][0][i] = rr[q];
        S.r[q][1][i] = ri[q];
      }
      __syncthreads();
    }
    ib = 1.0 / b;
    if (fac) fac[(2 * LOG) * NT + i] = ib;
  }
  // slopes
  __syncthreads();
#pragma unroll
  for (int q = 0; q < SB; ++q) {
    S.r[q][0][i] = rr[q] * ib;
    S.r[q][1][i] = ri[q] * ib;
  }
  __syncthreads();

  if (i < n) {
    const double h = S.sh[i], ih = 1.0 / h;
#pragma unroll
    for (int q = 0; q < SB; ++q) {
      if (q >= ns) break;
      const int series = s0 + q;
      const double2 y0v = series_value(series, i, K, y0, y1, y2, y3, A);
      const double2 y1v = series_value(series, i + 1, K, y0, y1, y2, y3, A);
      const double dr = (y1v.x - y0v.x) * ih, di = (y1v.y - y0v.y) * ih;
      const double s0r = S.r[q][0][i], s1r = S.r[q][0][i + 1], s0i = S.r[q][1][i], s1i = S.r[q][1][i + 1];
      const double c2r = (3.0 * dr - 2.0 * s0r - s1r) * ih;
      const double c3r = (s0r + s1r - 2.0 * dr) * ih * ih;
      if (series < 4) {
        double* o = tcoef + ((size_t)series * n + i) * 4;
        o[0] = y0v.x;
        o[1] = s0r;
        o[2] = c2r;
        o[3] = c3r;
      } else {
        const double c2i = (3.0 * di - 2.0 * s0i - s1i) * ih;
        const double c3i = (s0i + s1i - 2.0 * di) * ih * ih;
        double* o = acoef + ((size_t)(series - 4) * n + i) * 8;
        o[0] = y0v.x;
        o[1] = y0v.y;
        o[2] = s0r;
        o[3] = s0i;
        o[4] = c2r;
        o[5] = c2i;
        o[6] = c3r;
        o[7] = c3i;
        if (acoef32) {
          // the mixed path's FP32 coefficients in the normalised variable
          // u = tau / h: A(t_i + u h) = sum_k (a_k h^k) u^k
          const double h2 = h * h, h3 = h2 * h;
          float* o32 = acoef32 + ((size_t)(series - 4) * n + i) * 8;
          o32[0] = (float)y0v.x;
          o32[1] = (float)y0v.y;
          o32[2] = (float)(s0r * h);
          o32[3] = (float)(s0i * h);
          o32[4] = (float)(c2r * h2);
          o32[5] = (float)(c2i * h2);
          o32[6] = (float)(c3r * h3);
          o32[7] = (float)(c3i * h3);
        }
      }
    }
  }
}

}  // namespace fdemri
