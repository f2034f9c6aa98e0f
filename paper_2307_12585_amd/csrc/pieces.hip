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
#include <algorithm>
#include <climits>

#include "fdemri_internal.hpp"
#include "harmonics.hpp"
#include "search.hpp"
#include "spline_core.hpp"

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
  float4* modes32;  // (c_+, c_x) in FP32 for the mixed path, or NULL
  int2* mode_kr;
  Piece* pieces;
  int64_t* evals;  // [Nm]
  uint32_t* flag_word;
};

// Segment-local part of the piece walk for spline segment i of one voice,
// computed once: the monotonic sub-intervals between the interior turning
// points of F_V (at most three), the direction of F_V on each, the zero
// crossing inside each (bisection to full precision) and whether F_V is
// exactly 0 at an interior knot ending the segment.  Which of these become
// piece-closing events depends only on the direction before the segment
// (segment_events below).
struct Event {
  double tau, F;
  int seg;
};

struct SegScan {
  double u0[3], F0[3];  // start of each sub-interval and F_V there
  double zc[3];         // zero crossing inside sub-interval j (bit j of zc_mask)
  int dir[3];           // direction of F_V on sub-interval j (0: flat)
  int nsub, zc_mask;
  bool zero_end;        // F_V == 0 exactly at the interior knot ending the segment
  int last_dir;         // last non-zero direction inside the segment (0 if flat)
  double h;             // segment length
};

__device__ __forceinline__ void scan_segment(const PieceArgs& a, int i, double m, double n, SegScan& S) {
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
  // turning points: sign changes of a1 + 2 a2 u + 3 a3 u^2 inside (0, h), ascending
  double t0 = 0.0, t1 = 0.0;
  int ntp = 0;
  {
    const double A2 = 3.0 * a3, B2 = 2.0 * a2, C2 = a1;
    double r0 = 0.0, r1 = 0.0;
    int nr = 0;
    if (A2 == 0.0) {
      if (B2 != 0.0) {
        r0 = -C2 / B2;
        nr = 1;
      }
    } else {
      const double disc = B2 * B2 - 4.0 * A2 * C2;
      if (disc > 0.0) {
        const double sq = sqrt(disc);
        const double q = -0.5 * (B2 + (B2 >= 0.0 ? sq : -sq));
        r0 = q / A2;
        nr = 1;
        if (q != 0.0) {
          r1 = C2 / q;
          nr = 2;
        }
      }
    }
    const bool k0 = nr >= 1 && r0 > 0.0 && r0 < h;
    const bool k1 = nr >= 2 && r1 > 0.0 && r1 < h;
    if (k0 && k1) {
      t0 = fmin(r0, r1);
      t1 = fmax(r0, r1);
      ntp = 2;
    } else if (k0 || k1) {
      t0 = k0 ? r0 : r1;
      ntp = 1;
    }
  }
  S.h = h;
  S.nsub = ntp + 1;
  S.zc_mask = 0;
  S.last_dir = 0;
  double u0 = 0.0, Fu0 = F0;
#pragma unroll
  for (int j = 0; j < 3; ++j) {
    S.u0[j] = u0;
    S.F0[j] = Fu0;
    S.dir[j] = 0;
    S.zc[j] = 0.0;
    if (j <= ntp) {
      const bool last = (j == ntp);
      const double u = last ? h : (j == 0 ? t0 : t1);
      const double Fu = last ? F1 : poly(u);
      const int dir = (Fu > Fu0) ? 1 : ((Fu < Fu0) ? -1 : 0);
      S.dir[j] = dir;
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
        S.zc[j] = 0.5 * (lo + hi);
        S.zc_mask |= 1 << j;
      }
      if (dir != 0) S.last_dir = dir;
      u0 = u;
      Fu0 = Fu;
    }
  }
  S.zero_end = (F1 == 0.0 && i + 1 < nseg);
}

// Piece-closing events of a scanned segment, in order, given the last
// non-zero direction before it: a change of direction at a sub-interval
// start (which may be a knot), a zero crossing inside a sub-interval, and
// F_V = 0 exactly at an interior knot.  With emit == false only the events
// are counted; with emit == true they are written to ev[base + ...] (bounded
// by cap).
__device__ __forceinline__ int segment_events(const SegScan& S, int i, int cur_dir, bool emit, Event* ev, int base,
                                              int cap) {
  int cnt = 0;
  auto push = [&](double tau, double F) {
    if (emit && base + cnt < cap) ev[base + cnt] = Event{tau, F, i};
    ++cnt;
  };
#pragma unroll
  for (int j = 0; j < 3; ++j) {
    if (j < S.nsub) {
      const int dir = S.dir[j];
      if (dir != 0 && cur_dir != 0 && dir != cur_dir) push(S.u0[j], S.F0[j]);
      if ((S.zc_mask >> j) & 1) push(S.zc[j], 0.0);
      if (dir != 0) cur_dir = dir;
    }
  }
  if (S.zero_end) push(S.h, 0.0);  // the end of the last sub-interval is the knot t_{i+1}
  return cnt;
}

// Orders a wavefront's LDS writes before its later LDS reads when lanes
// exchange data through LDS (each wave owns its event buffer).
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
}

// Rows outside the harmonics' range (or, unless the caller lists both signs,
// with m < 0) contribute nothing and are flagged.
__device__ __forceinline__ bool rejected_row(int l, int m, uint32_t flags) {
  return l < 2 || l > kMaxL || m > l || m < -l || (m < 0 && !(flags & FDEMRI_NO_PARTNERS));
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
  // the grid's end values, for the bin-range searches at the end (requested
  // first, so that their latency overlaps the segment scan)
  const double fbeg = a.f[0], fend = a.f[a.Nf - 1];
  const int li = a.l[mu], mi = a.m[mu], ni = a.n[mu];
  const double m = (double)mi, n = (double)ni;
  const int K = a.K, nseg = K - 1;

  // ---- ordered events over all segments
  int n_ev = 0;           // events found so far (may exceed kMaxEvents)
  int carry_dir = 0;      // last non-zero direction before the current chunk
  const bool bad_mode = rejected_row(li, mi, a.flags);
  const bool flat_voice = (mi == 0 && ni == 0) || bad_mode;
  if (!flat_voice) {
    for (int c0 = 0; c0 < nseg; c0 += 64) {
      const int i = c0 + lane;
      SegScan S;
      S.nsub = 0;
      S.zc_mask = 0;
      S.zero_end = false;
      S.last_dir = 0;
      if (i < nseg) scan_segment(a, i, m, n, S);
      const int own_last = S.last_dir;
      const unsigned long long nz = __ballot(own_last != 0);
      const unsigned long long below = nz & ((1ull << lane) - 1ull);
      const int src = below ? 63 - __clzll((long long)below) : 0;
      const int from_below = __shfl(own_last, src, 64);
      const int incoming = below ? from_below : carry_dir;
      // events with the true incoming direction (count, then place)
      const int cnt = (i < nseg) ? segment_events(S, i, incoming, false, ev, 0, 0) : 0;
      int pre = cnt;  // inclusive prefix sum over lanes
#pragma unroll
      for (int off = 1; off < 64; off <<= 1) {
        const int v = __shfl_up(pre, off, 64);
        if (lane >= off) pre += v;
      }
      const int total = __shfl(pre, 63, 64);
      if (i < nseg && cnt > 0) segment_events(S, i, incoming, true, ev, n_ev + pre - cnt, kMaxEvents);
      n_ev += total;
      if (nz) carry_dir = __shfl(own_last, 63 - __clzll((long long)nz), 64);
    }
  }
  wave_lds_sync();
  // final event: the end of the trajectory
  const double Fend = knot_freq(m, a.Fphi[nseg], n, a.Fr[nseg]);
  const double hend = a.t[nseg] - a.t[nseg - 1];
  const bool ev_overflow = (n_ev + 1 > kMaxEvents);
  const int n_all = ev_overflow ? kMaxEvents : n_ev + 1;
  if (lane == 0) ev[min(n_ev, kMaxEvents - 1)] = Event{hend, Fend, nseg - 1};
  wave_lds_sync();

  // ---- pieces between consecutive events, one per lane
  const int kpos = first_gt(a.f, a.Nf, 0.0, fbeg, fend);  // first bin with f > 0 (wave-uniform)
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
      P.rate = (double)(P.seg_b - P.seg_a + 1) / (P.g_b - P.g_a);
      P.rate0 = (double)P.seg_a - P.rate * P.g_a;
      P.dd = (double)P.d;
      P.sd = (double)P.s;
      P.whole = (n_all == 1) ? 1 : 0;  // lane 0 from the first knot to the final event
      P.pad = 0;
      const double glo = fmin(P.g_a, P.g_b), ghi = fmax(P.g_a, P.g_b);
      int klo = first_ge(a.f, a.Nf, glo, fbeg, fend);
      if (klo < kpos) klo = kpos;
      P.k_lo = klo;
      P.k_hi = first_gt(a.f, a.Nf, ghi, fbeg, fend) - 1;
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

  // ---- fused polarization factors (harmonics by the whole wave)
  const double4 yy = swsh_m2_pair_wave(li, mi, a.theta, a.phi);
  if (lane == 0) {
    ModeConst mc;
    mc.m = m;
    mc.n = n;
    const double2 y = make_double2(yy.x, yy.y);
    double2 yp = make_double2(0.0, 0.0);  // (-1)^l conj Y_{l,-m}
    if (mi > 0 && !(a.flags & FDEMRI_NO_PARTNERS)) {
      const double sg = (li & 1) ? -1.0 : 1.0;
      yp = make_double2(sg * yy.z, -sg * yy.w);
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
    if (a.modes32) a.modes32[mu] = make_float4((float)mc.cp_re, (float)mc.cp_im, (float)mc.cx_re, (float)mc.cx_im);
    a.mode_kr[mu] = make_int2(kr_lo, kr_hi);
    a.evals[mu] = evals;
    if (n_valid > kMaxPieces || ev_overflow) atomicOr(a.flag_word, (uint32_t)FDEMRI_FLAG_PIECE_OVERFLOW);
    if (bad_mode) atomicOr(a.flag_word, (uint32_t)FDEMRI_FLAG_BAD_MODE);
  }
}

// ---- voice groups
// Rows are grouped by (m, n) through a 32-bit sort key: bits 31..25 hold
// m + 64, bits 24..13 n + 2048, bits 12..0 the row (kGroupMaxModes <= 2^13).
// A row that can join no group, because the set-up rejects it (it gets no
// pieces) or its n does not fit the 12-bit field, has the m-field kAlone and
// n-field 0: it sorts after every group and stays on its own.  Keys are
// distinct, so their order (the sort is not stable) is unique: members
// follow each other in row order and a group's first member is its lowest
// row.
static_assert(kGroupMaxModes <= 1 << 13, "row field of the group key");
constexpr uint32_t kAlone = 127u;

__device__ __forceinline__ uint32_t group_key(int l, int m, int n, uint32_t flags, int row) {
  if (rejected_row(l, m, flags) || n < -2048 || n > 2047) return (kAlone << 25) | (uint32_t)row;
  return ((uint32_t)(m + 64) << 25) | ((uint32_t)(n + 2048) << 13) | (uint32_t)row;
}

// Keys the sort of Nm rows holds: a power of two >= Nm, and at least two per
// thread.
__host__ __device__ inline int group_sort_size(int Nm, int NT) {
  int n2 = 2 * NT;
  while (n2 < Nm) n2 <<= 1;
  return n2;
}

__device__ __forceinline__ void compare_exchange(uint32_t& a, uint32_t& b, bool up) {
  const uint32_t lo = min(a, b), hi = max(a, b);
  a = up ? lo : hi;
  b = up ? hi : lo;
}

// Stage of stride S < KPL of the bitonic merge of blocks of `size` keys: both
// partners are in the thread's registers.
template <int KPL, int S>
__device__ __forceinline__ void sort_stage_in_lane(uint32_t (&k)[KPL], bool up_thread, int size) {
  if constexpr (S < KPL) {
#pragma unroll
    for (int q = 0; q < KPL; ++q) {
      if ((q & S) == 0) {
        // direction bit of position base + q: for blocks of fewer than KPL
        // keys it lies in q (a scalar test), otherwise in the thread's base
        const bool up = size < KPL ? (q & size) == 0 : up_thread;
        compare_exchange(k[q], k[q + S], up);
      }
    }
  }
}

// Sort of the rows' keys by one workgroup of NT threads, KPL keys per thread
// in registers (thread t holds positions t KPL .. t KPL + KPL - 1; n2 = NT KPL
// keys, padded with ~0): a bitonic network whose stages exchange partners
// within a thread's registers (stride < KPL), across the lanes of a wave
// (shuffles), or, for strides of a wave's keys or more, through LDS (lds, n2
// words).  Then, from the sorted keys, the group size at every first
// position of a group (0 elsewhere) into gsize and the row of every position
// into gmem[].mode.  The workgroup runs at raised wave priority: it shares
// its SIMDs with the set-up's other work, and the gather waits for it.
template <int NT, int KPL>
__device__ void group_sort_kpl(const int32_t* __restrict__ l, const int32_t* __restrict__ m,
                               const int32_t* __restrict__ n, uint32_t flags, int Nm, uint32_t* lds,
                               int32_t* __restrict__ gsize, GroupMember* __restrict__ gmem) {
  constexpr int N2 = NT * KPL, WK = 64 * KPL, NW = NT / 64;
  static_assert(N2 <= kGroupMaxModes && KPL <= 32, "sort size");
  __shared__ int wmin[NW];
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const int base = t * KPL;
  uint32_t k[KPL];
#pragma unroll
  for (int q = 0; q < KPL; ++q) {
    const int j = base + q;
    k[q] = j < Nm ? group_key(l[j], m[j], n[j], flags, j) : ~0u;
  }
  for (int size = 2; size <= N2; size <<= 1) {
    for (int s = size >> 1; s > 0; s >>= 1) {
      // with s and size at least KPL the partner and the direction bits lie
      // in the thread's base, the same for all its keys
      const bool keep_min = ((base & s) == 0) == ((base & size) == 0);
      if (s >= WK) {
        __syncthreads();  // the previous stage's readers are done
#pragma unroll
        for (int q = 0; q < KPL; ++q) lds[base + q] = k[q];
        __syncthreads();
        uint32_t o[KPL];
#pragma unroll
        for (int q = 0; q < KPL; ++q) o[q] = lds[(base + q) ^ s];
#pragma unroll
        for (int q = 0; q < KPL; ++q) k[q] = keep_min ? min(k[q], o[q]) : max(k[q], o[q]);
      } else if (s >= KPL) {
        // partner lane: lane ^ (s / KPL), same register; all the exchanges
        // are issued before any is used
        const int addr = (lane ^ (s / KPL)) << 2;
        uint32_t o[KPL];
#pragma unroll
        for (int q = 0; q < KPL; ++q) o[q] = (uint32_t)__builtin_amdgcn_ds_bpermute(addr, (int)k[q]);
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int q = 0; q < KPL; ++q) k[q] = keep_min ? min(k[q], o[q]) : max(k[q], o[q]);
      } else {
        const bool up_thread = (base & size) == 0;
        if (s == 1)
          sort_stage_in_lane<KPL, 1>(k, up_thread, size);
        else if (s == 2)
          sort_stage_in_lane<KPL, 2>(k, up_thread, size);
        else if (s == 4)
          sort_stage_in_lane<KPL, 4>(k, up_thread, size);
        else if (s == 8)
          sort_stage_in_lane<KPL, 8>(k, up_thread, size);
        else
          sort_stage_in_lane<KPL, 16>(k, up_thread, size);
      }
    }
  }
  // first positions of groups (a padding position counts as one)
  __syncthreads();
  lds[base + KPL - 1] = k[KPL - 1];  // each thread's last key, for its successor
  __syncthreads();
  uint32_t prev = base > 0 ? lds[base - 1] : 0u;
  uint32_t first = 0;
  int my_first = INT_MAX;
#pragma unroll
  for (int q = 0; q < KPL; ++q) {
    const int j = base + q;
    const bool f = j >= Nm || j == 0 || (k[q] >> 25) == kAlone || (prev >> 13) != (k[q] >> 13);
    if (f) {
      first |= 1u << q;
      my_first = min(my_first, j);
    }
    prev = k[q];
  }
  // the nearest first position after this thread's: a suffix minimum
  int v = my_first;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const int o = __shfl_down(v, off, 64);
    if (lane + off < 64) v = min(v, o);
  }
  if (lane == 0) wmin[wave] = v;
  int next = __shfl_down(v, 1, 64);
  if (lane == 63) next = INT_MAX;
  __syncthreads();
  for (int w = wave + 1; w < NW; ++w) next = min(next, wmin[w]);
  int e = min(next, Nm);
#pragma unroll
  for (int q = KPL - 1; q >= 0; --q) {
    const int j = base + q;
    const bool f = (first >> q) & 1u;
    if (j < Nm) {
      gsize[j] = f ? e - j : 0;
      gmem[j].mode = (int)(k[q] & (uint32_t)(kGroupMaxModes - 1));
    }
    if (f) e = j;
  }
}

// The voice groups' sort (gsize, gmem[].mode) of Nm rows by one workgroup of
// NT threads, LDS lds of group_sort_size(Nm, NT) words.
template <int NT>
__device__ void group_sort(const int32_t* __restrict__ l, const int32_t* __restrict__ m,
                           const int32_t* __restrict__ n, uint32_t flags, int Nm, uint32_t* lds,
                           int32_t* __restrict__ gsize, GroupMember* __restrict__ gmem) {
  __builtin_amdgcn_s_setprio(3);
  switch (group_sort_size(Nm, NT) / NT) {
    case 2:
      group_sort_kpl<NT, 2>(l, m, n, flags, Nm, lds, gsize, gmem);
      break;
    case 4:
      group_sort_kpl<NT, 4>(l, m, n, flags, Nm, lds, gsize, gmem);
      break;
    case 8:
      if constexpr (NT * 8 <= kGroupMaxModes) group_sort_kpl<NT, 8>(l, m, n, flags, Nm, lds, gsize, gmem);
      break;
    case 16:
      if constexpr (NT * 16 <= kGroupMaxModes) group_sort_kpl<NT, 16>(l, m, n, flags, Nm, lds, gsize, gmem);
      break;
    case 32:
      if constexpr (NT * 32 <= kGroupMaxModes) group_sort_kpl<NT, 32>(l, m, n, flags, Nm, lds, gsize, gmem);
      break;
  }
  __builtin_amdgcn_s_setprio(0);
}

// Position j of the voice groups, once the sort and the row's mode table are
// written: the group's bin range at its first position (empty elsewhere),
// the member's polarization factors (gsize[j] and gmem[j].mode are the
// sort's, and the mode field is not rewritten); returns the bin range
// written to gkr[j].
__device__ __forceinline__ int2 group_fill(int j, const ModeConst* __restrict__ modes,
                                           const float4* __restrict__ modes32, const int2* __restrict__ mode_kr,
                                           int2* __restrict__ gkr, const int32_t* __restrict__ gsize,
                                           GroupMember* __restrict__ gmem, GroupMember32* __restrict__ gmem32) {
  const int row = gmem[j].mode;
  const int2 kr = gsize[j] > 0 ? mode_kr[row] : make_int2(INT_MAX, -1);
  gkr[j] = kr;
  const ModeConst md = modes[row];
  double2* c = (double2*)&gmem[j];
  c[0] = make_double2(md.cp_re, md.cp_im);
  c[1] = make_double2(md.cx_re, md.cx_im);
  if (gmem32) gmem32[j] = GroupMember32{modes32[row], row, {0, 0, 0}};
  return kr;
}

// Combined amplitude splines of the voice group of g >= 2 rows at sorted
// position j, segment i: the coefficients of sum_t c+_t A_t and of
// sum_t cx_t A_t over its rows t (the spline of a weighted sum of series is
// the weighted sum of their splines, and the sum over a group's rows of
// c_t A_t(t(f)) E is (sum_t c_t A_t)(t(f)) E), which replace the segment's
// coefficients of the group's first and second row: in place in acoef (FP64
// path), or in their FP32 normalised form in acoef32 (mixed path; acoef is
// then left as it is).  The thread reads every row's coefficients of the
// segment before it writes.
__device__ __forceinline__ void combine_segment(int j, int g, int i, int nseg, double h,
                                                const ModeConst* __restrict__ modes,
                                                const GroupMember* __restrict__ gmem, double* __restrict__ acoef,
                                                float* __restrict__ acoef32) {
  constexpr int U = 4;  // rows whose loads are in flight together
  double P[8], X[8];
#pragma unroll
  for (int k = 0; k < 8; ++k) P[k] = X[k] = 0.0;
  for (int q0 = 0; q0 < g; q0 += U) {
    int row[U];
#pragma unroll
    for (int u = 0; u < U; ++u) row[u] = q0 + u < g ? gmem[j + q0 + u].mode : -1;
    double2 cp[U], cx[U];
    double a[U][8];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      if (row[u] >= 0) {
        const ModeConst& md = modes[row[u]];
        cp[u] = make_double2(md.cp_re, md.cp_im);
        cx[u] = make_double2(md.cx_re, md.cx_im);
        const double2* s = (const double2*)(acoef + ((size_t)row[u] * nseg + i) * 8);
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          const double2 v = s[k];
          a[u][2 * k] = v.x;
          a[u][2 * k + 1] = v.y;
        }
      } else {
        cp[u] = cx[u] = make_double2(0.0, 0.0);
#pragma unroll
        for (int k = 0; k < 8; ++k) a[u][k] = 0.0;
      }
    }
    // in row order (the zero terms of absent rows change nothing)
#pragma unroll
    for (int u = 0; u < U; ++u) {
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const double ar = a[u][2 * k], ai = a[u][2 * k + 1];
        P[2 * k] += cp[u].x * ar - cp[u].y * ai;
        P[2 * k + 1] += cp[u].x * ai + cp[u].y * ar;
        X[2 * k] += cx[u].x * ar - cx[u].y * ai;
        X[2 * k + 1] += cx[u].x * ai + cx[u].y * ar;
      }
    }
  }
  const size_t sp = ((size_t)gmem[j].mode * nseg + i) * 8, sx = ((size_t)gmem[j + 1].mode * nseg + i) * 8;
  if (acoef32) {
    amp32_segment(P, h, acoef32 + sp);
    amp32_segment(X, h, acoef32 + sx);
  } else {
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      acoef[sp + k] = P[k];
      acoef[sx + k] = X[k];
    }
  }
}

// Bin envelope [env[0], env[1]] of one waveform's voices (min and max over
// the non-empty per-mode ranges; {INT_MAX, -1} when all are empty), by one
// workgroup of kGroupThreads threads.  The gather skips the blocks outside
// the envelope without reading the mode table.
constexpr int kGroupThreads = 1024;

// Minimum of lo and maximum of hi over a workgroup of NT threads (valid in
// thread 0).
template <int NT>
__device__ __forceinline__ void block_min_max(int& lo, int& hi) {
  constexpr int NW = NT / 64;
  __shared__ int s_lo[NW], s_hi[NW];
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) {
    lo = min(lo, __shfl_xor(lo, off, 64));
    hi = max(hi, __shfl_xor(hi, off, 64));
  }
  if ((threadIdx.x & 63) == 0) {
    s_lo[threadIdx.x >> 6] = lo;
    s_hi[threadIdx.x >> 6] = hi;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 1; w < NW; ++w) {
      lo = min(lo, s_lo[w]);
      hi = max(hi, s_hi[w]);
    }
  }
}

__device__ void envelope_block(const int2* __restrict__ mode_kr, int Nm, int32_t* __restrict__ env) {
  int lo = INT_MAX, hi = -1;
  for (int mu = threadIdx.x; mu < Nm; mu += kGroupThreads) {
    const int2 r = mode_kr[mu];
    if (r.x <= r.y) {
      lo = min(lo, r.x);
      hi = max(hi, r.y);
    }
  }
  block_min_max<kGroupThreads>(lo, hi);
  if (threadIdx.x == 0) {
    env[0] = lo;
    env[1] = hi;
  }
}

// One waveform's envelope (more than kGroupMaxModes rows: not grouped).
__global__ __launch_bounds__(kGroupThreads) void envelope_kernel(const int2* __restrict__ mode_kr, int Nm,
                                                                 int32_t* __restrict__ env) {
  envelope_block(mode_kr, Nm, env);
}

// One grouped waveform after its set-up launch.  The first fill_blocks
// workgroups, one position per thread: the groups' tables and the envelope,
// as the minimum and maximum over the groups' ranges into env (set to
// {INT_MAX, -1} by the sort).  The rest, one (position, segment) per thread:
// the combined amplitude splines of the groups of two or more rows (with
// acoef not NULL).
constexpr int kFillThreads = 256;
__global__ __launch_bounds__(kFillThreads) void group_fill_kernel(const ModeConst* __restrict__ modes,
                                                                  const float4* __restrict__ modes32,
                                                                  const int2* __restrict__ mode_kr, int Nm,
                                                                  int32_t* __restrict__ env, int2* gkr,
                                                                  const int32_t* gsize, GroupMember* gmem,
                                                                  GroupMember32* gmem32, int fill_blocks, int nseg,
                                                                  const double* __restrict__ t, double* acoef,
                                                                  float* acoef32) {
  if ((int)blockIdx.x >= fill_blocks) {
    const int q = ((int)blockIdx.x - fill_blocks) * kFillThreads + (int)threadIdx.x;
    const int j = q / nseg, i = q - j * nseg;
    if (j >= Nm) return;
    const int g = gsize[j];
    if (g >= 2) combine_segment(j, g, i, nseg, t[i + 1] - t[i], modes, gmem, acoef, acoef32);
    return;
  }
  const int j = (int)blockIdx.x * kFillThreads + (int)threadIdx.x;
  int lo = INT_MAX, hi = -1;
  if (j < Nm) {
    const int2 kr = group_fill(j, modes, modes32, mode_kr, gkr, gsize, gmem, gmem32);
    if (kr.x <= kr.y) {
      lo = kr.x;
      hi = kr.y;
    }
  }
  block_min_max<kFillThreads>(lo, hi);
  if (threadIdx.x == 0 && lo <= hi) {
    atomicMin(&env[0], lo);
    atomicMax(&env[1], hi);
  }
}

// Batched: one workgroup per waveform, which also sorts the rows of a
// grouped waveform.
__global__ __launch_bounds__(kGroupThreads) void envelope_batch_kernel(const WaveItem* __restrict__ items) {
  __shared__ uint32_t key[kGroupMaxModes];
  const WaveItem& w = items[blockIdx.x];
  envelope_block(w.mode_kr, w.Nm, w.status + 1);
  if (!w.gkr) return;
  group_sort<kGroupThreads>(w.l, w.m, w.n, w.flags, w.Nm, key, w.gsize, w.gmem);
  __syncthreads();  // the sort's gsize and gmem[].mode, written to global memory
  for (int j = threadIdx.x; j < w.Nm; j += kGroupThreads)
    group_fill(j, w.modes, w.modes32, w.mode_kr, w.gkr, w.gsize, w.gmem, w.gmem32);
  // the combined amplitude splines (the mixed path writes the FP32 form)
  const int nseg = w.K - 1;
  for (int q = threadIdx.x; q < w.Nm * nseg; q += kGroupThreads) {
    const int j = q / nseg, i = q - j * nseg;
    const int g = w.gsize[j];
    if (g >= 2) combine_segment(j, g, i, nseg, w.t[i + 1] - w.t[i], w.modes, w.gmem, w.acoef, w.acoef32);
  }
}

// Inputs of one waveform's checks (device pointers of the caller's arrays).
struct CheckArgs {
  int32_t K, Nm, Nf;
  uint32_t flags;
  int hann;  // the grid must be f_k = k f_1 (the 3-tap Hann kernel's DFT grid)
  const double *t, *Fphi, *Fr, *Phiphi, *Phir, *A, *f;
};

// Workgroup blk of the checks of one waveform (check_blocks of them): 0 the
// trajectory (t finite and strictly increasing, the frequencies and phases
// finite), then the amplitude array in chunks (finite), then the frequency
// grid in chunks (finite, >= 0, ascending; with hann also |f_k - k f_1| <=
// 1e-12 f_k, so f_0 = 0).  Failures set bits in the waveform's status word
// and the context's flag bit; nothing is written otherwise.  With slot, the
// workgroup instead writes its result to *slot (0 when its part passed),
// every time.
__device__ void check_block(const CheckArgs& c, int blk, int32_t* status, uint32_t* flag_word,
                            int32_t* slot = nullptr) {
  constexpr int U = 4;
  int32_t bad = 0;
  const long na = check_amp_count(c.K, c.Nm, c.flags);
  const int nab = (int)((na + kCheckChunk - 1) / kCheckChunk);
  if (blk == 0) {
    for (int i = threadIdx.x; i < c.K; i += blockDim.x) {
      const double ti = c.t[i];
      if (!isfinite(ti) || (i > 0 && !(ti > c.t[i - 1]))) bad |= kBadKnots;
      if (!isfinite(c.Fphi[i]) || !isfinite(c.Fr[i]) || !isfinite(c.Phiphi[i]) || !isfinite(c.Phir[i]))
        bad |= kBadValues;
    }
  } else if (blk <= nab) {
    // U elements per thread and round, their loads issued together
    const long base = (long)(blk - 1) * kCheckChunk;
    for (int j0 = 0; j0 < kCheckChunk; j0 += U * (int)blockDim.x) {
      double v[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const long e = base + j0 + u * (int)blockDim.x + threadIdx.x;
        v[u] = e < na ? c.A[e] : 0.0;
      }
#pragma unroll
      for (int u = 0; u < U; ++u)
        if (!isfinite(v[u])) bad |= kBadValues;
    }
  } else {
    const long base = (long)(blk - 1 - nab) * kCheckChunk;
    const double f1 = c.Nf > 1 ? c.f[1] : 0.0;
    for (int j0 = 0; j0 < kCheckChunk; j0 += U * (int)blockDim.x) {
      double v[U], prev[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const long k = base + j0 + u * (int)blockDim.x + threadIdx.x;
        v[u] = k < c.Nf ? c.f[k] : 0.0;
        prev[u] = (k > 0 && k < c.Nf) ? c.f[k - 1] : 0.0;
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const long k = base + j0 + u * (int)blockDim.x + threadIdx.x;
        if (k < c.Nf) {
          const double fk = v[u];
          if (!isfinite(fk) || !(fk >= 0.0) || (k > 0 && !(fk >= prev[u]))) bad |= kBadGrid;
          if (c.hann && !(fabs(fk - (double)k * f1) <= 1e-12 * fk)) bad |= kBadHannGrid;
        }
      }
    }
  }
  if (slot) {
    __shared__ int s_bad;
    if (threadIdx.x == 0) s_bad = 0;
    __syncthreads();
    if (bad) atomicOr(&s_bad, bad);
    __syncthreads();
    if (threadIdx.x == 0) {
      *slot = s_bad;
      if (s_bad) atomicOr(flag_word, (uint32_t)FDEMRI_FLAG_BAD_INPUT);
    }
    return;
  }
  if (bad) {
    atomicOr(status, bad);
    atomicOr(flag_word, (uint32_t)FDEMRI_FLAG_BAD_INPUT);
  }
}

// Batched pieces: one wavefront per mode, kPieceWaves modes per workgroup.
constexpr int kPieceWaves = 4;

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
  a.modes32 = w.modes32;
  a.mode_kr = w.mode_kr;
  a.pieces = w.pieces;
  a.evals = w.evals;
  a.flag_word = flag_word;
  return a;
}

// Index b of the prefix array pre[0..B] with pre[b] <= g < pre[b + 1].
__device__ __forceinline__ int prefix_find(const int32_t* __restrict__ pre, int B, int g) {
  int lo = 0, hi = B - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (pre[mid] <= g)
      lo = mid;
    else
      hi = mid - 1;
  }
  return lo;
}

// Batched: the first piece_blocks workgroups run one wavefront per (waveform,
// mode) through the prefix of Nm_b; the rest run the input checks of every
// waveform through the prefix of its check_blocks (check_prefix).
__global__ __launch_bounds__(64 * kPieceWaves) void pieces_batch_kernel(const WaveItem* __restrict__ items, int B,
                                                                        const int32_t* __restrict__ mode_prefix,
                                                                        int total, int piece_blocks,
                                                                        const int32_t* __restrict__ check_prefix,
                                                                        int hann, uint32_t* flag_word) {
  __shared__ Event ev[kPieceWaves][kMaxEvents];
  if ((int)blockIdx.x >= piece_blocks) {
    const int g = (int)blockIdx.x - piece_blocks;
    const int b = prefix_find(check_prefix, B, g);
    const WaveItem& w = items[b];
    const CheckArgs c{w.K, w.Nm, w.Nf, w.flags, hann, w.t, w.Fphi, w.Fr, w.Phiphi, w.Phir, w.A, w.f};
    check_block(c, g - check_prefix[b], w.status, flag_word);
    return;
  }
  const int wave = threadIdx.x >> 6;
  const int g = blockIdx.x * kPieceWaves + wave;
  if (g >= total) return;
  const int lo = prefix_find(mode_prefix, B, g);
  const PieceArgs a = piece_args_of(items[lo], flag_word);
  piece_mode_wave(a, g - mode_prefix[lo], ev[wave]);
}

// The batch's piece tables and its input checks in one launch (total_checks:
// the sum of the waveforms' check_blocks; hann: the likelihood's Hann kernel
// needs DFT grids), then the waveforms' bin envelopes.
hipError_t launch_pieces_batch(const WaveItem* items, int B, const int32_t* mode_prefix, int total_modes,
                               const int32_t* check_prefix, int total_checks, int hann, uint32_t* flag_word,
                               hipStream_t stream) {
  const int blocks = (total_modes + kPieceWaves - 1) / kPieceWaves;
  pieces_batch_kernel<<<blocks + total_checks, 64 * kPieceWaves, 0, stream>>>(
      items, B, mode_prefix, total_modes, blocks, check_prefix, hann, flag_word);
  envelope_batch_kernel<<<B, kGroupThreads, 0, stream>>>(items);
  return hipGetLastError();
}

// Set-up of one waveform after its trajectory splines: the piece tables (one
// wave per mode), the amplitude splines (kSeriesPerBlock modes per
// workgroup, all sharing the knot matrix; with acoef32 also their FP32 form)
// and the input checks in one launch, the pieces' workgroups first.  The two parts are independent, so the amplitude
// splines fill the machine while the latency-bound piece walks run, instead
// of taking a launch of their own before them.
template <int NT>
__global__ __launch_bounds__(NT) void setup_kernel(PieceArgs a, int piece_blocks, int amp_blocks,
                                                   const double* __restrict__ A, double* __restrict__ acoef,
                                                   float* __restrict__ acoef32, double* fac, CheckArgs c,
                                                   int32_t* __restrict__ status, int32_t* __restrict__ gsize,
                                                   GroupMember* __restrict__ gmem, int32_t* __restrict__ env) {
  constexpr int W = NT / 64;
  // LDS (setup_lds_bytes) of any part: the spline's tables, the waves' event
  // buffers or the sort's keys
  extern __shared__ double lds[];
  int b = (int)blockIdx.x;
  if (gsize) {
    // workgroup 0 sorts the rows into voice groups, concurrently with the rest
    if (b == 0) {
      if (threadIdx.x == 0) {
        env[0] = INT_MAX;  // for the fill's atomics
        env[1] = -1;
      }
      group_sort<NT>(a.l, a.m, a.n, a.flags, a.Nm, (uint32_t*)lds, gsize, gmem);
      return;
    }
    --b;
  }
  if (b < piece_blocks) {
    const int wave = threadIdx.x >> 6;
    const int mu = b * W + wave;
    if (mu < a.Nm) piece_mode_wave(a, mu, (Event*)lds + wave * kMaxEvents);
    return;
  }
  if (b >= piece_blocks + amp_blocks) {
    check_block(c, b - piece_blocks - amp_blocks, status, a.flag_word);
    return;
  }
  const int s0 = 4 + (b - piece_blocks) * kSeriesPerBlock;
  // series 4 + mu only (the trajectory arguments are never read here), with
  // the knot matrix's reduction factors from the trajectory splines
  spline_block<NT, true>(*(SplineLds<NT>*)lds, s0, 4 + a.Nm, a.K, a.t, a.Fphi, a.Fr, a.Fphi, a.Fr, A, acoef, acoef,
                         fac, acoef32);
}

// Dynamic LDS of setup_kernel<NT> (with the sort of Nm rows when grouped).
template <int NT>
size_t setup_lds_bytes(int Nm, bool grouped) {
  constexpr size_t W = NT / 64;
  size_t bytes = sizeof(SplineLds<NT>) > sizeof(Event) * W * kMaxEvents ? sizeof(SplineLds<NT>)
                                                                         : sizeof(Event) * W * kMaxEvents;
  if (grouped) bytes = std::max(bytes, sizeof(uint32_t) * (size_t)group_sort_size(Nm, NT));
  return bytes;
}

// The piece tables, unless A is NULL the amplitude splines of Nm modes
// (acoef [Nm][K-1][8]; with acoef32 also the FP32 normalised form, and the
// FP32 mode constants in modes32), and the input checks (A_in: the caller's
// amplitude array, knot values or coefficients; hann: the grid must be the
// Hann kernel's DFT grid), in one launch; then, for more than
// kEnvelopeMinModes modes, the bin envelope and (modes_grouped) the voice
// groups in gkr, gsize, gmem and gmem32 (mixed).  The trajectory
// spline coefficients tcoef and the knot matrix's reduction factors fac,
// written by launch_spline with the same thread count, must be in place
// (stream order).
hipError_t launch_setup_flat(int K, int Nm, int Nf, const double* t, const double* Fphi, const double* Fr,
                             const double* f, const double* tcoef, const int32_t* l, const int32_t* m,
                             const int32_t* n, double theta, double phi, double scale, uint32_t flags,
                             const double* A, double* acoef, float* acoef32, double* fac, ModeConst* modes,
                             float4* modes32, int2* mode_kr, Piece* pieces, int64_t* evals, int32_t* status,
                             uint32_t* flag_word, const double* Phiphi, const double* Phir, const double* A_in,
                             int hann, bool grouped, bool combine, int2* gkr, int32_t* gsize, GroupMember* gmem,
                             GroupMember32* gmem32, hipStream_t stream) {
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
  a.modes32 = modes32;
  a.mode_kr = mode_kr;
  a.pieces = pieces;
  a.evals = evals;
  a.flag_word = flag_word;
  const int amp_blocks = A ? (Nm + kSeriesPerBlock - 1) / kSeriesPerBlock : 0;
  const int checks = check_blocks(K, Nm, Nf, flags);
  const CheckArgs c{K, Nm, Nf, flags, hann, t, Fphi, Fr, Phiphi, Phir, A_in, f};
  const int sb = grouped ? 1 : 0;  // the sort's workgroup
  int32_t* sort_gsize = grouped ? gsize : nullptr;
  if (K <= 256) {
    const int pb = (Nm + 3) / 4;
    setup_kernel<256><<<sb + pb + amp_blocks + checks, 256, setup_lds_bytes<256>(Nm, grouped), stream>>>(
        a, pb, amp_blocks, A, acoef, acoef32, fac, c, status, sort_gsize, gmem, status + 1);
  } else {
    const int pb = (Nm + 7) / 8;
    setup_kernel<512><<<sb + pb + amp_blocks + checks, 512, setup_lds_bytes<512>(Nm, grouped), stream>>>(
        a, pb, amp_blocks, A, acoef, acoef32, fac, c, status, sort_gsize, gmem, status + 1);
  }
  // a large mode table gets its bin envelope (and, up to kGroupMaxModes
  // rows, its voice groups from the set-up's sort, one position per thread),
  // so that the gather skips the blocks no voice reaches without scanning the
  // table and solves each root once per group; a small table is scanned as
  // cheaply as the launch would cost
  if (grouped) {
    const int fill_blocks = (Nm + kFillThreads - 1) / kFillThreads;
    const int pairs = Nm * (K - 1);  // at most kGroupMaxModes (kMaxKnots - 1)
    const int combine_blocks = combine ? (pairs + kFillThreads - 1) / kFillThreads : 0;
    group_fill_kernel<<<fill_blocks + combine_blocks, kFillThreads, 0, stream>>>(
        modes, modes32, mode_kr, Nm, status + 1, gkr, gsize, gmem, gmem32, fill_blocks, K - 1, t, acoef, acoef32);
  }
  else if (Nm > kEnvelopeMinModes)
    envelope_kernel<<<1, kGroupThreads, 0, stream>>>(mode_kr, Nm, status + 1);
  return hipGetLastError();
}

// Fused set-up of a small waveform (kFusedMax* limits), one launch in place
// of the trajectory splines' launch and setup_kernel's: the piece workgroups
// first solve the splines of F_phi and F_r themselves (the same arithmetic as
// the spline launch, so the same coefficients, which each writes to tcoef),
// then walk their modes; one workgroup solves those of Phi_phi and Phi_r;
// the amplitude workgroups reduce the knot matrix themselves instead of
// reading its factors; the check workgroups write one status slot each.
template <int NT>
__global__ __launch_bounds__(NT) void setup_fused_kernel(PieceArgs a, int piece_blocks, int amp_blocks,
                                                         const double* __restrict__ A, double* __restrict__ acoef,
                                                         float* __restrict__ acoef32, double* __restrict__ tcoef,
                                                         const double* __restrict__ Phiphi,
                                                         const double* __restrict__ Phir, CheckArgs c,
                                                         int32_t* __restrict__ slots) {
  constexpr int W = NT / 64;
  constexpr size_t kBytes = sizeof(SplineLds<NT>) > sizeof(Event) * W * kMaxEvents ? sizeof(SplineLds<NT>)
                                                                                     : sizeof(Event) * W * kMaxEvents;
  __shared__ double lds[kBytes / sizeof(double)];
  const int b = (int)blockIdx.x;
  if (b < piece_blocks) {
    // series 0 and 1 (F_phi, F_r) into tcoef, read back by this workgroup's
    // piece walks (every piece workgroup writes the same values)
    spline_block<NT>(*(SplineLds<NT>*)lds, 0, 4, a.K, a.t, a.Fphi, a.Fr, Phiphi, Phir, A, tcoef, acoef);
    __syncthreads();  // the coefficients are written, the LDS free
    const int wave = threadIdx.x >> 6;
    const int mu = b * W + wave;
    if (mu < a.Nm) piece_mode_wave(a, mu, (Event*)lds + wave * kMaxEvents);
    return;
  }
  if (b == piece_blocks) {
    spline_block<NT>(*(SplineLds<NT>*)lds, 2, 4, a.K, a.t, a.Fphi, a.Fr, Phiphi, Phir, A, tcoef, acoef);
    return;
  }
  if (b > piece_blocks + amp_blocks) {
    const int blk = b - piece_blocks - amp_blocks - 1;
    check_block(c, blk, nullptr, a.flag_word, slots + blk);
    return;
  }
  const int s0 = 4 + (b - piece_blocks - 1) * kSeriesPerBlock;
  spline_block<NT>(*(SplineLds<NT>*)lds, s0, 4 + a.Nm, a.K, a.t, a.Fphi, a.Fr, a.Fphi, a.Fr, A, acoef, acoef,
                   nullptr, acoef32);
}

// Whether the set-up of a waveform of this shape can be fused (and then
// how many status slots it writes: check_blocks).
bool setup_fusable(int K, int Nm, int Nf, uint32_t flags) {
  return Nm <= kFusedMaxModes && K <= kFusedMaxKnots && check_blocks(K, Nm, Nf, flags) <= kFusedMaxSlots;
}

// The fused set-up (setup_fused_kernel) of a waveform for which setup_fusable
// holds: as launch_spline followed by launch_setup_flat, with the input
// statuses in slots[check_blocks] instead of the status word.
hipError_t launch_setup_fused(int K, int Nm, int Nf, const double* t, const double* Fphi, const double* Fr,
                              const double* Phiphi, const double* Phir, const double* f, double* tcoef,
                              const int32_t* l, const int32_t* m, const int32_t* n, double theta, double phi,
                              double scale, uint32_t flags, const double* A, double* acoef, float* acoef32,
                              ModeConst* modes, float4* modes32, int2* mode_kr, Piece* pieces, int64_t* evals,
                              int32_t* slots, uint32_t* flag_word, const double* A_in, int hann,
                              hipStream_t stream) {
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
  a.modes32 = modes32;
  a.mode_kr = mode_kr;
  a.pieces = pieces;
  a.evals = evals;
  a.flag_word = flag_word;
  const int amp_blocks = A ? (Nm + kSeriesPerBlock - 1) / kSeriesPerBlock : 0;
  const int checks = check_blocks(K, Nm, Nf, flags);
  const CheckArgs c{K, Nm, Nf, flags, hann, t, Fphi, Fr, Phiphi, Phir, A_in, f};
  const int pb = (Nm + 3) / 4;
  setup_fused_kernel<256><<<pb + 1 + amp_blocks + checks, 256, 0, stream>>>(a, pb, amp_blocks, A, acoef, acoef32,
                                                                            tcoef, Phiphi, Phir, c, slots);
  return hipGetLastError();
}

}  // namespace fdemri
