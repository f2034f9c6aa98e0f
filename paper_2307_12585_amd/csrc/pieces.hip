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

// Segment-local part of the piece walk for spline segment i of one voice:
// the monotonic sub-intervals between the interior turning points, and the
// piece-closing events in order.  A piece closes where the direction of F_V
// changes (at a sub-interval start, which may be a knot), where F_V changes
// sign inside a sub-interval (bisection to full precision), and where F_V is
// exactly 0 at an interior knot.  `cur_dir` is the last non-zero direction
// before the segment.  With emit == false only the events are counted; with
// emit == true they are written to ev[base + ...] (bounded by cap).  Returns
// the number of events and, in last_dir, the last non-zero direction inside
// the segment (0 if F_V is flat on it).
struct Event {
  double tau, F;
  int seg;
};

__device__ int segment_events(const PieceArgs& a, int i, double m, double n, int cur_dir, bool emit, Event* ev,
                              int base, int cap, int& last_dir) {
  const int nseg = a.K - 1;
  const double h = a.t[i + 1] - a.t[i];
  const double* cp_ = a.tcoef + (size_t)i * 4;
  const double* cr_ = a.tcoef + ((size_t)nseg + i) * 4;
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
  int cnt = 0;
  last_dir = 0;
  auto push = [&](double tau, double F) {
    if (emit && base + cnt < cap) ev[base + cnt] = Event{tau, F, i};
    ++cnt;
  };
  double u0 = 0.0, Fu0 = F0;
  for (int j = 0; j <= ntp; ++j) {
    const bool last = (j == ntp);
    const double u = last ? h : tp[j];
    const double Fu = last ? F1 : poly(u);
    const int dir = (Fu > Fu0) ? 1 : ((Fu < Fu0) ? -1 : 0);
    if (dir != 0 && cur_dir != 0 && dir != cur_dir) push(u0, Fu0);
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
      push(0.5 * (lo + hi), 0.0);
    }
    if (dir != 0) {
      cur_dir = dir;
      last_dir = dir;
    }
    if (last && Fu == 0.0 && i + 1 < nseg) push(u, 0.0);  // F_V = 0 exactly at an interior knot
    u0 = u;
    Fu0 = Fu;
  }
  return cnt;
}

// Mode constants and monotonic pieces of one voice, computed by one full
// wavefront: lanes walk 64 spline segments at a time; the running direction
// is carried across segments by a ballot scan, the events are compacted in
// order into LDS, and the pieces between consecutive events are built (bin
// ranges by binary search) one per lane.  Equivalent to walking the
// segments one by one: a piece spans consecutive events and is kept when its
// end frequencies differ.
constexpr int kMaxEvents = 64;

__device__ void piece_mode_wave(const PieceArgs& a, const int mu, Event* ev) {
  const int lane = threadIdx.x & 63;
  const int li = a.l[mu], mi = a.m[mu], ni = a.n[mu];
  const double m = (double)mi, n = (double)ni;
  const int K = a.K, nseg = K - 1;

  // ---- ordered events over all segments
  int n_ev = 0;           // events found so far (may exceed kMaxEvents)
  int carry_dir = 0;      // last non-zero direction before the current chunk
  const bool flat_voice = (mi == 0 && ni == 0);
  if (!flat_voice) {
    for (int c0 = 0; c0 < nseg; c0 += 64) {
      const int i = c0 + lane;
      int own_last = 0, cnt = 0;
      // pass 1: own last direction (independent of the incoming direction)
      if (i < nseg) {
        int ld;
        segment_events(a, i, m, n, 0, false, ev, 0, 0, ld);
        own_last = ld;
      }
      const unsigned long long nz = __ballot(own_last != 0);
      const unsigned long long below = nz & ((1ull << lane) - 1ull);
      const int src = below ? 63 - __clzll((long long)below) : 0;
      const int from_below = __shfl(own_last, src, 64);
      const int incoming = below ? from_below : carry_dir;
      // pass 2: events with the true incoming direction (count, then place)
      int ld = 0;
      if (i < nseg) cnt = segment_events(a, i, m, n, incoming, false, ev, 0, 0, ld);
      int pre = cnt;  // inclusive prefix sum over lanes
#pragma unroll
      for (int off = 1; off < 64; off <<= 1) {
        const int v = __shfl_up(pre, off, 64);
        if (lane >= off) pre += v;
      }
      const int total = __shfl(pre, 63, 64);
      if (i < nseg && cnt > 0) segment_events(a, i, m, n, incoming, true, ev, n_ev + pre - cnt, kMaxEvents, ld);
      n_ev += total;
      if (nz) carry_dir = __shfl(own_last, 63 - __clzll((long long)nz), 64);
    }
  }
  __syncthreads();
  // final event: the end of the trajectory
  const double Fend = knot_freq(m, a.Fphi[nseg], n, a.Fr[nseg]);
  const double hend = a.t[nseg] - a.t[nseg - 1];
  const bool ev_overflow = (n_ev + 1 > kMaxEvents);
  const int n_all = ev_overflow ? kMaxEvents : n_ev + 1;
  if (lane == 0) ev[min(n_ev, kMaxEvents - 1)] = Event{hend, Fend, nseg - 1};
  __syncthreads();

  // ---- pieces between consecutive events, one per lane
  const int kpos = upper_bound(a.f, a.Nf, 0.0);  // first bin with f > 0 (wave-uniform)
  const int n_cand = flat_voice ? 0 : n_all;
  bool valid = false;
  Piece P{};
  if (lane < n_cand) {
    const Event eb = ev[lane];
    Event ea;
    if (lane == 0)
      ea = Event{0.0, knot_freq(m, a.Fphi[0], n, a.Fr[0]), 0};
    else
      ea = ev[lane - 1];
    if (eb.F != ea.F) {
      valid = true;
      const int s = (ea.F + eb.F > 0.0) ? 1 : -1;
      const int dV = (eb.F > ea.F) ? 1 : -1;
      P.seg_a = ea.seg;
      P.tau_a = ea.tau;
      P.seg_b = eb.seg;
      P.tau_b = eb.tau;
      P.g_a = s * ea.F;
      P.g_b = s * eb.F;
      P.s = s;
      P.d = s * dV;
      P.rate = (float)((double)(P.seg_b - P.seg_a + 1) / (P.g_b - P.g_a));
      P.pad1 = 0;
      const double glo = fmin(P.g_a, P.g_b), ghi = fmax(P.g_a, P.g_b);
      int klo = lower_bound(a.f, a.Nf, glo);
      if (klo < kpos) klo = kpos;
      P.k_lo = klo;
      P.k_hi = upper_bound(a.f, a.Nf, ghi) - 1;
    }
  }
  const unsigned long long vmask = __ballot(valid);
  const int idx = __popcll(vmask & ((1ull << lane) - 1ull));
  const int n_valid = __popcll(vmask);
  Piece* out = a.pieces + (size_t)mu * kMaxPieces;
  int64_t evals = 0;
  int kr_lo = INT_MAX, kr_hi = -1;
  if (valid && idx < kMaxPieces) {
    out[idx] = P;
    if (P.k_lo <= P.k_hi) {
      evals = (int64_t)(P.k_hi - P.k_lo + 1);
      kr_lo = P.k_lo;
      kr_hi = P.k_hi;
    }
  }
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) {
    evals += __shfl_xor(evals, off, 64);
    kr_lo = min(kr_lo, __shfl_xor(kr_lo, off, 64));
    kr_hi = max(kr_hi, __shfl_xor(kr_hi, off, 64));
  }

  if (lane == 0) {
    // ---- fused polarization factors
    ModeConst mc;
    mc.m = m;
    mc.n = n;
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
    mc.npieces = min(n_valid, kMaxPieces);
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
    if (n_valid > kMaxPieces || ev_overflow) atomicOr(a.flag_word, (uint32_t)FDEMRI_FLAG_PIECE_OVERFLOW);
  }
}

// One wavefront per mode.
__global__ __launch_bounds__(64) void pieces_kernel(PieceArgs a) {
  __shared__ Event ev[kMaxEvents];
  piece_mode_wave(a, blockIdx.x, ev);
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

// Batched: one wavefront per (waveform, mode) through the prefix of Nm_b.
__global__ __launch_bounds__(64) void pieces_batch_kernel(const WaveItem* __restrict__ items, int B,
                                                          const int32_t* __restrict__ mode_prefix, int total,
                                                          uint32_t* flag_word) {
  __shared__ Event ev[kMaxEvents];
  const int g = blockIdx.x;
  int lo = 0, hi = B - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (mode_prefix[mid] <= g)
      lo = mid;
    else
      hi = mid - 1;
  }
  const PieceArgs a = piece_args_of(items[lo], flag_word);
  piece_mode_wave(a, g - mode_prefix[lo], ev);
}

hipError_t launch_pieces_batch(const WaveItem* items, int B, const int32_t* mode_prefix, int total_modes,
                               uint32_t* flag_word, hipStream_t stream) {
  pieces_batch_kernel<<<total_modes, 64, 0, stream>>>(items, B, mode_prefix, total_modes, flag_word);
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
  pieces_kernel<<<Nm, 64, 0, stream>>>(a);
  return hipGetLastError();
}

}  // namespace fdemri
