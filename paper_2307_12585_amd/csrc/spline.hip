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
// The tridiagonal system is solved by parallel cyclic reduction, one
// workgroup per series with one thread per knot, so that every series is
// solved in log2(K) LDS steps instead of a K-long serial recursion.  Each
// segment then gets the Hermite coefficients
//   c0 = y_i, c1 = s_i, c2 = (3 delta_i - 2 s_i - s_{i+1})/h_i,
//   c3 = (s_i + s_{i+1} - 2 delta_i)/h_i^2.
#include "fdemri_internal.hpp"

namespace fdemri {

template <int NT>
struct SplineLds {
  double sa[NT], sb[NT], sc[NT], sr[NT], si[NT];
  double sy_re[NT], sy_im[NT], sh[NT];
};

// One series (0..3 trajectory, real; 4 + mode: complex amplitude) of one
// waveform, solved by the NT threads of the calling workgroup.
template <int NT>
__device__ void spline_series(SplineLds<NT>& S, int series, int K, const double* __restrict__ t,
                              const double* __restrict__ y0, const double* __restrict__ y1,
                              const double* __restrict__ y2, const double* __restrict__ y3,
                              const double* __restrict__ A, double* __restrict__ tcoef, double* __restrict__ acoef) {
  double* sa = S.sa;
  double* sb = S.sb;
  double* sc = S.sc;
  double* sr = S.sr;
  double* si = S.si;
  double* sy_re = S.sy_re;
  double* sy_im = S.sy_im;
  double* sh = S.sh;
  const int i = threadIdx.x;
  const bool cplx = series >= 4;
  const int mode = series - 4;
  const int n = K - 1;  // segments

  // load knots
  if (i < K) {
    double yr, yi = 0.0;
    if (!cplx) {
      const double* y = series == 0 ? y0 : series == 1 ? y1 : series == 2 ? y2 : y3;
      yr = y[i];
    } else {
      const double* a = A + ((size_t)mode * K + i) * 2;
      yr = a[0];
      yi = a[1];
    }
    sy_re[i] = yr;
    sy_im[i] = yi;
  }
  if (i < n) sh[i] = t[i + 1] - t[i];
  __syncthreads();
  if (K > NT) return;  // the host never launches this; keeps every index below in bounds

  // assemble row i
  double a = 0.0, b = 1.0, c = 0.0, rr = 0.0, ri = 0.0;
  if (i < K) {
    auto delta = [&](int j, double& dr, double& di) {
      dr = (sy_re[j + 1] - sy_re[j]) / sh[j];
      di = (sy_im[j + 1] - sy_im[j]) / sh[j];
    };
    if (i == 0) {
      double h0 = sh[0], h1 = sh[1], d0r, d0i, d1r, d1i;
      delta(0, d0r, d0i);
      delta(1, d1r, d1i);
      double w = 1.0 / (h0 + h1);
      a = 0.0;
      b = h1;
      c = h0 + h1;
      rr = ((2.0 * h1 * h1 + 3.0 * h0 * h1) * d0r + h0 * h0 * d1r) * w;
      ri = ((2.0 * h1 * h1 + 3.0 * h0 * h1) * d0i + h0 * h0 * d1i) * w;
    } else if (i == n) {
      double hm = sh[n - 2], hl = sh[n - 1], dmr, dmi, dlr, dli;
      delta(n - 2, dmr, dmi);
      delta(n - 1, dlr, dli);
      double w = 1.0 / (hm + hl);
      a = hm + hl;
      b = hm;
      c = 0.0;
      rr = (hl * hl * dmr + (2.0 * hm * hm + 3.0 * hm * hl) * dlr) * w;
      ri = (hl * hl * dmi + (2.0 * hm * hm + 3.0 * hm * hl) * dli) * w;
    } else {
      double hp = sh[i - 1], hi = sh[i], dpr, dpi, dir_, dii;
      delta(i - 1, dpr, dpi);
      delta(i, dir_, dii);
      a = hi;
      b = 2.0 * (hp + hi);
      c = hp;
      rr = 3.0 * (hi * dpr + hp * dir_);
      ri = 3.0 * (hi * dpi + hp * dii);
    }
  }
  sa[i] = a;
  sb[i] = b;
  sc[i] = c;
  sr[i] = rr;
  si[i] = ri;
  __syncthreads();

  // parallel cyclic reduction: after step j every row couples only to rows +-2^(j+1)
  for (int s = 1; s < NT; s <<= 1) {
    const int im = i - s, ip = i + s;
    double am = 0.0, bm = 1.0, cm = 0.0, rm = 0.0, qm = 0.0;
    double ap = 0.0, bp = 1.0, cp = 0.0, rp = 0.0, qp = 0.0;
    if (im >= 0) {
      am = sa[im];
      bm = sb[im];
      cm = sc[im];
      rm = sr[im];
      qm = si[im];
    }
    if (ip < NT) {
      ap = sa[ip];
      bp = sb[ip];
      cp = sc[ip];
      rp = sr[ip];
      qp = si[ip];
    }
    const double k1 = a / bm, k2 = c / bp;
    const double na = -am * k1;
    const double nc = -cp * k2;
    const double nb = b - cm * k1 - ap * k2;
    const double nr = rr - rm * k1 - rp * k2;
    const double ni = ri - qm * k1 - qp * k2;
    __syncthreads();
    a = na;
    b = nb;
    c = nc;
    rr = nr;
    ri = ni;
    sa[i] = a;
    sb[i] = b;
    sc[i] = c;
    sr[i] = rr;
    si[i] = ri;
    __syncthreads();
  }
  // slopes
  const double s_re = rr / b, s_im = ri / b;
  __syncthreads();
  sr[i] = s_re;
  si[i] = s_im;
  __syncthreads();

  if (i < n) {
    const double h = sh[i], ih = 1.0 / h;
    const double dr = (sy_re[i + 1] - sy_re[i]) * ih, di = (sy_im[i + 1] - sy_im[i]) * ih;
    const double s0r = sr[i], s1r = sr[i + 1], s0i = si[i], s1i = si[i + 1];
    const double c2r = (3.0 * dr - 2.0 * s0r - s1r) * ih;
    const double c3r = (s0r + s1r - 2.0 * dr) * ih * ih;
    if (!cplx) {
      double* o = tcoef + ((size_t)series * n + i) * 4;
      o[0] = sy_re[i];
      o[1] = s0r;
      o[2] = c2r;
      o[3] = c3r;
    } else {
      const double c2i = (3.0 * di - 2.0 * s0i - s1i) * ih;
      const double c3i = (s0i + s1i - 2.0 * di) * ih * ih;
      double* o = acoef + ((size_t)mode * n + i) * 8;
      o[0] = sy_re[i];
      o[1] = sy_im[i];
      o[2] = s0r;
      o[3] = s0i;
      o[4] = c2r;
      o[5] = c2i;
      o[6] = c3r;
      o[7] = c3i;
    }
  }
}

template <int NT>
__global__ __launch_bounds__(NT) void spline_pcr_kernel(int K, const double* __restrict__ t,
                                                        const double* __restrict__ y0, const double* __restrict__ y1,
                                                        const double* __restrict__ y2, const double* __restrict__ y3,
                                                        const double* __restrict__ A, int Nm, double* __restrict__ tcoef,
                                                        double* __restrict__ acoef) {
  __shared__ SplineLds<NT> S;
  spline_series<NT>(S, blockIdx.x, K, t, y0, y1, y2, y3, A, tcoef, acoef);
}

// Batched: block -> (waveform, series) through the prefix of 4 + Nm_b.
template <int NT>
__global__ __launch_bounds__(NT) void spline_batch_kernel(const WaveItem* __restrict__ items, int B,
                                                          const int32_t* __restrict__ series_prefix) {
  __shared__ SplineLds<NT> S;
  const int g = blockIdx.x;
  int lo = 0, hi = B - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (series_prefix[mid] <= g)
      lo = mid;
    else
      hi = mid - 1;
  }
  const WaveItem& w = items[lo];
  spline_series<NT>(S, g - series_prefix[lo], w.K, w.t, w.Fphi, w.Fr, w.Phiphi, w.Phir, w.A, w.tcoef, w.acoef);
}

// Host launcher: coefficients of the four trajectory series and of Nm
// complex amplitude series, all on knots t[K].
hipError_t launch_spline(int K, const double* t, const double* Fphi, const double* Fr, const double* Phiphi,
                         const double* Phir, const double* A, int Nm, double* tcoef, double* acoef,
                         hipStream_t stream) {
  dim3 grid(4 + Nm);
  if (K <= 64)
    spline_pcr_kernel<64><<<grid, 64, 0, stream>>>(K, t, Fphi, Fr, Phiphi, Phir, A, Nm, tcoef, acoef);
  else if (K <= 128)
    spline_pcr_kernel<128><<<grid, 128, 0, stream>>>(K, t, Fphi, Fr, Phiphi, Phir, A, Nm, tcoef, acoef);
  else if (K <= 256)
    spline_pcr_kernel<256><<<grid, 256, 0, stream>>>(K, t, Fphi, Fr, Phiphi, Phir, A, Nm, tcoef, acoef);
  else
    spline_pcr_kernel<512><<<grid, 512, 0, stream>>>(K, t, Fphi, Fr, Phiphi, Phir, A, Nm, tcoef, acoef);
  return hipGetLastError();
}

hipError_t launch_spline_batch(const WaveItem* items, int B, const int32_t* series_prefix, int total_series, int Kmax,
                               hipStream_t stream) {
  dim3 grid(total_series);
  if (Kmax <= 64)
    spline_batch_kernel<64><<<grid, 64, 0, stream>>>(items, B, series_prefix);
  else if (Kmax <= 128)
    spline_batch_kernel<128><<<grid, 128, 0, stream>>>(items, B, series_prefix);
  else if (Kmax <= 256)
    spline_batch_kernel<256><<<grid, 256, 0, stream>>>(items, B, series_prefix);
  else
    spline_batch_kernel<512><<<grid, 512, 0, stream>>>(items, B, series_prefix);
  return hipGetLastError();
}

}  // namespace fdemri
