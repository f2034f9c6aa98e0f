// Per-mode set-up before the summation (Sec. 2.2): the fused polarization
// factors of each (l,m,n) voice and the table of monotonic pieces of its
// frequency F_V(t) = m F_phi(t) + n F_r(t) (k = 0 for Schwarzschild).
//
// Sec. 2.2 solves the cubic of Eq. cubic_equation inside the spline segment
// that holds f, with one or two real roots per segment when F_V turns over.
// Here every voice is instead cut once, before the summation, at the zeros
// of dF_V/dt (turnovers) and of F_V (sign changes), into pieces on which
// |F_V| is monotonic.  Each bin then has at most one root per piece, the
// root set over all pieces equals the set of real roots inside the
// trajectory, and the summation kernel only needs a bracketed solve.
//
// Polarizations: for a table row (l, m > 0, n) the voices (l,m,n) and
// (l,-m,-n) (amplitude (-1)^l conj A) both enter h = h_+ - i h_x
// (Eq. main_wave).  With the transform of Eq. singlevoiceFT,
// h_+(f) = [h(f) + conj h(-f)]/2 and h_x(f) = i[h(f) - conj h(-f)]/2, and the
// contributions of both voices at one root combine into
//   h_+ += (A c_+)^(s) E,  h_x += (A c_x)^(s) E,
//   c_+ = scale/2 (Y_lm + (-1)^l conj Y_{l,-m}),  c_x = i scale/2 (Y_lm - (-1)^l conj Y_{l,-m}),
// where (.)^(s) conjugates on pieces with F_V < 0 and
// E = e^{i(2 pi f t - s Phi_V)} G(s dF_V/dt, s d2F_V/dt2) for the root t.
#include <climits>

#include "fdemri_internal.hpp"
#include "harmonics.hpp"

namespace fdemri {

struct PieceArgs {
  int32_t K, Nm, Nf;
  const double* t;
  const double* Fphi;
  const double* Fr;
  const double* f;
  const double* tcoef;  // [4][K-1][4]
  const int32_t* l;
  const int32_t* m;
  const int32_t* n;
  double theta, phi, scale;
  uint32_t flags;
  ModeConst* modes;
  int2* mode_kr;
  Piece* pieces;
  int64_t* evals;  // [Nm]
  int32_t* env;    // [2]
  uint32_t* flag_word;
};

// first index k with f[k] >= x (f ascending), in [0, Nf]
__device__ __forceinline__ int lower_bound(const double* f, int Nf, double x) {
  int lo = 0, hi = Nf;
  while (lo < hi) {
    int mid = (lo + hi) >> 1;
    if (f[mid] < x)
      lo = mid + 1;
    else
      hi = mid;
  }
  return lo;
}

// first index k with f[k] > x
__device__ __forceinline__ int upper_bound(const double* f, int Nf, double x) {
  int lo = 0, hi = Nf;
  while (lo < hi) {
    int mid = (lo + hi) >> 1;
    if (f[mid] <= x)
      lo = mid + 1;
    else
      hi = mid;
  }
  return lo;
}

__device__ void piece_mode(const PieceArgs& a, const int mu) {
  const int li = a.l[mu], mi = a.m[mu], ni = a.n[mu];
  const double m = (double)mi, n = (double)ni;

  // ---- fused polarization factors
  ModeConst mc;
  mc.m = m;
  mc.n = n;
  {
    const double2 y = swsh_m2(li, mi, a.theta, a.phi);
    double2 yp = make_double2(0.0, 0.0);  // (-1)^l conj Y_{l,-m}
    if (mi > 0 && !(a.flags & FDEMRI_NO_PARTNERS)) {
      const double2 ym = swsh_m2(li, -mi, a.theta, a.phi);
      const double sg = (li & 1) ? -1.0 : 1.0;
      yp = make_double2(sg * ym.x, -sg * ym.y);
    }
    const double hs = 0.5 * a.scale;
    mc.cp_re = hs * (y.x + yp.x);
    mc.cp_im = hs * (y.y + yp.y);
    // i (y - yp) = (-(y.y - yp.y), y.x - yp.x)
    mc.cx_re = -hs * (y.y - yp.y);
    mc.cx_im = hs * (y.x - yp.x);
  }

  // ---- monotonic pieces of F_V
  const int K = a.K, nseg = K - 1;
  const double* t = a.t;
  const double* cFp = a.tcoef;                   // series 0
  const double* cFr = a.tcoef + (size_t)nseg * 4;  // series 1
  const int kpos = upper_bound(a.f, a.Nf, 0.0);  // first bin with f > 0
  Piece* out = a.pieces + (size_t)mu * kMaxPieces;
  int np = 0;
  bool overflow = false;
  int64_t evals = 0;
  int kr_lo = INT_MAX, kr_hi = -1;

  int sa = 0;
  double ta = 0.0;
  double Fa = knot_freq(m, a.Fphi[0], n, a.Fr[0]);

  auto close_piece = [&](int sb, double tb, double Fb) {
    if (Fb != Fa) {
      Piece P;
      const int s = (Fa + Fb > 0.0) ? 1 : -1;
      const int dV = (Fb > Fa) ? 1 : -1;
      P.seg_a = sa;
      P.tau_a = ta;
      P.seg_b = sb;
      P.tau_b = tb;
      P.g_a = s * Fa;
      P.g_b = s * Fb;
      P.s = s;
      P.d = s * dV;
      P.pad0 = P.pad1 = 0;
      const double glo = fmin(P.g_a, P.g_b), ghi = fmax(P.g_a, P.g_b);
      int klo = lower_bound(a.f, a.Nf, glo);
      if (klo < kpos) klo = kpos;
      const int khi = upper_bound(a.f, a.Nf, ghi) - 1;
      P.k_lo = klo;
      P.k_hi = khi;
      if (np < kMaxPieces) {
        out[np++] = P;
        if (klo <= khi) {
          evals += (int64_t)(khi - klo + 1);
          kr_lo = min(kr_lo, klo);
          kr_hi = max(kr_hi, khi);
        }
      } else {
        overflow = true;
      }
    }
    sa = sb;
    ta = tb;
    Fa = Fb;
  };

  if (!(mi == 0 && ni == 0)) {
    int cur_dir = 0;  // direction of F_V on the open piece (0: not known yet)
    for (int i = 0; i < nseg; ++i) {
      const double h = t[i + 1] - t[i];
      const double* cp_ = cFp + (size_t)i * 4;
      const double* cr_ = cFr + (size_t)i * 4;
      const double F0 = knot_freq(m, a.Fphi[i], n, a.Fr[i]);
      const double F1 = knot_freq(m, a.Fphi[i + 1], n, a.Fr[i + 1]);
      const double a1 = m * cp_[1] + n * cr_[1];
      const double a2 = m * cp_[2] + n * cr_[2];
      const double a3 = m * cp_[3] + n * cr_[3];
      auto poly = [&](double u) { return F0 + u * (a1 + u * (a2 + u * a3)); };
      // turning points: sign changes of a1 + 2 a2 u + 3 a3 u^2 inside (0, h)
      double tp[2];
      int ntp = 0;
      {
        const double A2 = 3.0 * a3, B2 = 2.0 * a2, C2 = a1;
        if (A2 == 0.0) {
          if (B2 != 0.0) tp[ntp++] = -C2 / B2;
        } else {
          const double disc = B2 * B2 - 4.0 * A2 * C2;
          if (disc > 0.0) {
            const double sq = sqrt(disc);
            const double q = -0.5 * (B2 + (B2 >= 0.0 ? sq : -sq));
            tp[ntp++] = q / A2;
            if (q != 0.0) tp[ntp++] = C2 / q;
          }
        }
        int keep = 0;
        for (int j = 0; j < ntp; ++j)
          if (tp[j] > 0.0 && tp[j] < h) tp[keep++] = tp[j];
        ntp = keep;
        if (ntp == 2 && tp[1] < tp[0]) {
          const double x = tp[0];
          tp[0] = tp[1];
          tp[1] = x;
        }
      }
      // walk the monotonic sub-intervals; a piece ends where F_V changes
      // sign (zero crossing) or where the direction of F_V changes (a
      // turnover inside a segment or exactly at a knot)
      double u0 = 0.0, Fu0 = F0;
      for (int j = 0; j <= ntp; ++j) {
        const bool last = (j == ntp);
        const double u = last ? h : tp[j];
        const double Fu = last ? F1 : poly(u);
        const int dir = (Fu > Fu0) ? 1 : ((Fu < Fu0) ? -1 : 0);
        if (dir != 0 && cur_dir != 0 && dir != cur_dir) close_piece(i, u0, Fu0);
        if ((Fu0 < 0.0 && Fu > 0.0) || (Fu0 > 0.0 && Fu < 0.0)) {
          // zero crossing inside the monotonic sub-interval (u0, u): bisection
          double lo = u0, hi = u, flo = Fu0;
          for (int it = 0; it < 200; ++it) {
            const double mid = 0.5 * (lo + hi);
            if (mid <= lo || mid >= hi) break;
            const double fm = poly(mid);
            if ((fm < 0.0) == (flo < 0.0)) {
              lo = mid;
              flo = fm;
            } else {
              hi = mid;
            }
          }
          close_piece(i, 0.5 * (lo + hi), 0.0);
        }
        if (dir != 0) cur_dir = dir;
        if (last && Fu == 0.0 && i + 1 < nseg) close_piece(i, u, 0.0);  // F_V = 0 exactly at a knot
        u0 = u;
        Fu0 = Fu;
      }
    }
    close_piece(nseg - 1, t[nseg] - t[nseg - 1], knot_freq(m, a.Fphi[nseg], n, a.Fr[nseg]));
  }

  mc.npieces = np;
  mc.pad = 0;
  mc.k_lo = kr_lo;
  mc.k_hi = kr_hi;
  a.modes[mu] = mc;
  a.mode_kr[mu] = make_int2(kr_lo, kr_hi);
  a.evals[mu] = evals;
  if (kr_lo <= kr_hi) {
    atomicMin(&a.env[0], kr_lo);
    atomicMax(&a.env[1], kr_hi);
  }
  if (overflow) atomicOr(a.flag_word, (uint32_t)FDEMRI_FLAG_PIECE_OVERFLOW);
}

__global__ __launch_bounds__(64) void pieces_kernel(PieceArgs a) {
  const int mu = blockIdx.x * blockDim.x + threadIdx.x;
  if (mu >= a.Nm) return;
  piece_mode(a, mu);
}

__device__ PieceArgs piece_args_of(const WaveItem& w, uint32_t* flag_word) {
  PieceArgs a;
  a.K = w.K;
  a.Nm = w.Nm;
  a.Nf = w.Nf;
  a.t = w.t;
  a.Fphi = w.Fphi;
  a.Fr = w.Fr;
  a.f = w.f;
  a.tcoef = w.tcoef;
  a.l = w.l;
  a.m = w.m;
  a.n = w.n;
  a.theta = w.theta;
  a.phi = w.phi;
  a.scale = w.scale;
  a.flags = w.flags;
  a.modes = w.modes;
  a.mode_kr = w.mode_kr;
  a.pieces = w.pieces;
  a.evals = w.evals;
  a.env = w.env;
  a.flag_word = flag_word;
  return a;
}

// Batched: thread -> (waveform, mode) through the prefix of Nm_b.
__global__ __launch_bounds__(64) void pieces_batch_kernel(const WaveItem* __restrict__ items, int B,
                                                          const int32_t* __restrict__ mode_prefix, int total,
                                                          uint32_t* flag_word) {
  const int g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= total) return;
  int lo = 0, hi = B - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (mode_prefix[mid] <= g)
      lo = mid;
    else
      hi = mid - 1;
  }
  const PieceArgs a = piece_args_of(items[lo], flag_word);
  piece_mode(a, g - mode_prefix[lo]);
}

hipError_t launch_pieces_batch(const WaveItem* items, int B, const int32_t* mode_prefix, int total_modes,
                               uint32_t* flag_word, hipStream_t stream) {
  const int threads = 64;
  pieces_batch_kernel<<<(total_modes + threads - 1) / threads, threads, 0, stream>>>(items, B, mode_prefix,
                                                                                     total_modes, flag_word);
  return hipGetLastError();
}

hipError_t launch_pieces_flat(int K, int Nm, int Nf, const double* t, const double* Fphi, const double* Fr,
                              const double* f, const double* tcoef, const int32_t* l, const int32_t* m,
                              const int32_t* n, double theta, double phi, double scale, uint32_t flags,
                              ModeConst* modes, int2* mode_kr, Piece* pieces, int64_t* evals, int32_t* env,
                              uint32_t* flag_word, hipStream_t stream) {
  PieceArgs a;
  a.K = K;
  a.Nm = Nm;
  a.Nf = Nf;
  a.t = t;
  a.Fphi = Fphi;
  a.Fr = Fr;
  a.f = f;
  a.tcoef = tcoef;
  a.l = l;
  a.m = m;
  a.n = n;
  a.theta = theta;
  a.phi = phi;
  a.scale = scale;
  a.flags = flags;
  a.modes = modes;
  a.mode_kr = mode_kr;
  a.pieces = pieces;
  a.evals = evals;
  a.env = env;
  a.flag_word = flag_word;
  const int threads = 64;
  const int blocks = (Nm + threads - 1) / threads;
  pieces_kernel<<<blocks, threads, 0, stream>>>(a);
  return hipGetLastError();
}

}  // namespace fdemri
