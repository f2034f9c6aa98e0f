// Frequency-domain mode sum (Sec. 2.2, Eqs. cubic_equation, SPAintegral2,
// extendedspa1), bin-major.
//
// The paper's GPU kernel places one block per (voice, spline segment) and
// adds every contribution atomically into the output vector.  Here each
// wavefront owns tiles of 64 contiguous frequency bins instead and gathers
// all contributions to its bins in registers, so every output element is
// written once, coalesced, in a fixed order of voices and pieces
// (deterministic, no atomics):
//   1. the workgroup lists, in LDS, the modes whose bin range meets its block
//      of bins and, if there are any, stages the shared trajectory tables
//      (knots and spline coefficients of F_phi, F_r, Phi_phi, Phi_r) in LDS
//      (a block no voice reaches only writes zeros);
//   2. for each listed mode and each of its monotonic pieces with bins in the
//      tile, each lane with a bin inside the piece's range finds the spline
//      segment holding f, solves the cubic of Eq. cubic_equation for the root
//      (secant start, safeguarded Halley steps), evaluates d|F|/dt,
//      d2|F|/dt2, the factor G of Eq. extendedspa1, the phase
//      2 pi f t - Phi_V(t) (large part in double-double, reduced modulo 2 pi)
//      and the amplitude spline, and accumulates h_+ and h_x;
//   3. the wave stores its tile.
// FP64 path: everything in double.  Mixed path: root, derivatives, phase and
// its reduction in double; the special function, sincos, amplitude spline and
// products in float, each contribution added to a double accumulator (fewer
// instructions than compensated float sums, at least as accurate).
#include <climits>

#include "evalcore.hpp"

namespace fdemri {

// Destination of the sums of a tile: the waveform (h_+, h_x per bin, complex128
// or complex64) or the partial sums of the Whittle log-likelihood
// (Eqs. likelihood and innerprod) against data d_p, d_c (same element type as
// the waveform) with per-bin weights wS = 4 w_k / S_n(f_k): per tile,
// partial[3] = (sum wS |d - h|^2, sum wS |h|^2, sum wS Re(conj(d) h)) over
// both channels and, with the 3-tap Hann kernel (hann != 0), the model at
// lanes 0, 1, 62 and 63 in edge[4][4], from which the terms of each tile's
// first and last bin are completed afterwards.
struct Sink {
  void* hp;
  void* hc;
  const void* d_p;
  const void* d_c;
  const double* wS;
  double* partial;
  double* edge;
  int hann;
};

// amp: the amplitude spline coefficients the path reads, [Nm][K-1][8]: the
// FP64 ones (p.acoef) or, on the mixed path, the FP32 normalised-u ones.  A
// field of its own, so that the kernel does not keep the whole table of
// trajectory pointers in registers for it.
struct GatherArgs {
  Prepared p;
  const void* amp;
  Sink out;
};

template <bool MIXED>
struct Acc;

template <>
struct Acc<false> {
  double v[4];
  __device__ __forceinline__ void zero() { v[0] = v[1] = v[2] = v[3] = 0.0; }
};

template <>
struct Acc<true> {
  double v[4];
  __device__ __forceinline__ void zero() { v[0] = v[1] = v[2] = v[3] = 0.0; }
  __device__ __forceinline__ void add(int q, float y) { v[q] += (double)y; }
};

// LDS copy of one waveform's trajectory tables, interleaved so that one base
// address per index reaches every field by immediate offsets: per knot i
// {F_phi, F_r, t, Phi_phi mod 2 pi, Phi_r mod 2 pi, h = t_{i+1} - t_i}
// (48 B, 16-B aligned pairs), per segment i the c1..c3 spline coefficients of
// F_phi, F_r, Phi_phi, Phi_r (96 B).
struct alignas(16) KnotRec {
  double Fp, Fr, t, Pp, Pr, h;
};
struct alignas(16) SegCoef {
  double cFp[3], cFr[3], cPp[3], cPr[3];
};
static_assert(sizeof(KnotRec) == 48 && sizeof(SegCoef) == 96, "LDS record layout");

// LDS address space for the device pass (the host pass has none).
#if defined(__HIP_DEVICE_COMPILE__)
#define klds __attribute__((address_space(3)))
#else
#define klds
#endif

// The tables as LDS pointers, so that addresses are 32-bit; a record's
// address is formed with a 24-bit multiply-add (indices stay below 2^24),
// which runs at full rate where a 32- or 64-bit integer multiply does not.
struct Lds {
  const klds KnotRec* kn;  // [K]
  const klds SegCoef* sc;  // [K-1]
  __device__ __forceinline__ const klds KnotRec& knot(int i) const {
    return *(const klds KnotRec*)((const klds char*)kn + __umul24(i, (int)sizeof(KnotRec)));
  }
  __device__ __forceinline__ const klds SegCoef& seg(int i) const {
    return *(const klds SegCoef*)((const klds char*)sc + __umul24(i, (int)sizeof(SegCoef)));
  }
};

// Secant steps on the segment index of a piece: at most this many, the first
// in every lane, the others in the lanes whose segment still fails the check
// while any lane of the wave does (dense inspirals, whose knot frequencies
// crowd at one end of the piece, need two to four; a slowly chirping voice
// one).
constexpr int kSecantSteps = 4;

// The members of a voice group as the evaluation reads them: with gm (and
// gm32 on the mixed path) the g rows of a sorted group, else the one row
// `mode` with the factors cP, cX (c32).
template <bool MIXED>
struct Members {
  const kconst GroupMember* gm;
  const kconst GroupMember32* gm32;
  int g;
  int mode;
  double2 cP, cX;
  float4 c32;
};

// The amplitude coefficients of row `mode` (wave-uniform: its base is scalar
// arithmetic) at segment i (a 32-bit byte offset from that base: one shift).
template <bool MIXED>
struct AmpOf;
template <>
struct AmpOf<false> {
  using T = AmpSeg64;
  __device__ __forceinline__ static T load(const void* __restrict__ amp, int nseg, int mode, int i) {
    const char* base = (const char*)amp + (size_t)mode * (size_t)nseg * 64;
    return load_amp64((const double*)(base + ((uint32_t)i << 6)));
  }
};
template <>
struct AmpOf<true> {
  using T = AmpSeg32;
  __device__ __forceinline__ static T load(const void* __restrict__ amp, int nseg, int mode, int i) {
    const char* base = (const char*)amp + (size_t)mode * (size_t)nseg * 32;
    return load_amp32((const float*)(base + ((uint32_t)i << 5)));
  }
};

// One (bin, piece) evaluation of a voice group.  The spline segment holding f
// is the largest i in [seg_a, seg_b] whose start value precedes f in the
// direction of the piece (i == seg_a or d g_i < d f; ties go to the lower
// segment).  It is guessed from the piece's rate, refined by secant steps on
// the segment index through the knot frequencies at the current segment, and
// checked against the definition; the rare misses walk to the right segment.
// The root and E = e^{i psi} G are formed once; a single row adds
// cP (A^(s) E) and cX (A^(s) E) with its amplitude spline A at the root
// (A^(s): A conjugated when s < 0), a group of two or more rows the same sum
// over its rows through its combined splines: (sum_t cP_t A_t)^(s) E and
// (sum_t cX_t A_t)^(s) E.
//   f, w: the bin frequency and 2 pi f;
//   ms, ns: s m and s n of the piece, so that |F_V| = ms F_phi + ns F_r;
//   neg: s < 0 (the factors of the members are then conjugated).
template <bool MIXED>
__device__ __forceinline__ void eval_bin(const double f, const double w, const Piece& P, const double ms, const double ns,
                                         const bool neg, const Members<MIXED>& M, const void* __restrict__ amp,
                                         int nseg, const Lds& L, Acc<MIXED>& acc) {
  const double dd_ = P.dd;
  const double fd = dd_ * f;
  // the conversion saturates (and takes NaN to 0); the clamp keeps the guess
  // inside the piece
  int i = min(max(cvt_i32_sat(__builtin_fma(f, P.rate, P.rate0)), P.seg_a), P.seg_b);
  double G0 = knot_freq(ms, L.knot(i).Fp, ns, L.knot(i).Fr);
  double G1 = knot_freq(ms, L.knot(i + 1).Fp, ns, L.knot(i + 1).Fr);
  auto secant = [&]() {
    const float num = (float)(f - G0);
    const float den = (float)(G1 - G0);
    float di = 0.f;
    // the step is bounded by the largest segment count, which keeps i + di
    // inside the int range
    constexpr float kStepMax = (float)kMaxKnots;
    if (den != 0.f) di = fminf(fmaxf(floorf(num * __builtin_amdgcn_rcpf(den)), -kStepMax), kStepMax);
    const int j = min(max(i + (int)di, P.seg_a), P.seg_b);
    if (j != i) {
      i = j;
      G0 = knot_freq(ms, L.knot(i).Fp, ns, L.knot(i).Fr);
      G1 = knot_freq(ms, L.knot(i + 1).Fp, ns, L.knot(i + 1).Fr);
    }
  };
  auto misses = [&]() { return (i > P.seg_a && !(dd_ * G0 < fd)) || (i < P.seg_b && dd_ * G1 < fd); };
  secant();
  bool miss = misses();
#pragma unroll 1
  for (int it = 1; it < kSecantSteps && __any(miss); ++it) {
    if (miss) {
      secant();
      miss = misses();
    }
  }
  if (miss) {
    while (i > P.seg_a && !(dd_ * knot_freq(ms, L.knot(i).Fp, ns, L.knot(i).Fr) < fd)) --i;
    while (i < P.seg_b && dd_ * knot_freq(ms, L.knot(i + 1).Fp, ns, L.knot(i + 1).Fr) < fd) ++i;
    G0 = knot_freq(ms, L.knot(i).Fp, ns, L.knot(i).Fr);
    G1 = knot_freq(ms, L.knot(i + 1).Fp, ns, L.knot(i + 1).Fr);
  }
  // the amplitude coefficients, requested now so that the load is in flight
  // during the root solve: a group of two or more rows has its combined
  // splines (sum_t c+_t A_t, sum_t cx_t A_t) in its first two rows' slots, a
  // single row its own
  const bool combined = M.g >= 2;
  const int mode0 = M.gm ? M.gm[0].mode : M.mode;
  using Seg = typename AmpOf<MIXED>::T;
  const Seg a0 = AmpOf<MIXED>::load(amp, nseg, mode0, i);
  SegData S;
  const klds KnotRec& kr = L.knot(i);
  S.ti = kr.t;
  S.h = kr.h;
  S.G0 = G0;
  S.G1 = G1;
  const klds SegCoef& cs = L.seg(i);
  S.q1 = wsum(ms, cs.cFp[0], ns, cs.cFr[0]);
  S.q2 = wsum(ms, cs.cFp[1], ns, cs.cFr[1]);
  S.q3 = wsum(ms, cs.cFp[2], ns, cs.cFr[2]);
  S.r1 = wsum(ms, cs.cPp[0], ns, cs.cPr[0]);
  S.r2 = wsum(ms, cs.cPp[1], ns, cs.cPr[1]);
  S.r3 = wsum(ms, cs.cPp[2], ns, cs.cPr[2]);
  S.Ppi = kr.Pp;
  S.Pri = kr.Pr;
  const Bracket B = make_bracket(P, i, S);
  const double tau = solve_root(f, dd_, S, B);
  // the second row's slot after the solve (both in flight across it would
  // spill registers); the phase and factor then cover its latency
  Seg a1{};
  if (combined) a1 = AmpOf<MIXED>::load(amp, nseg, M.gm[1].mode, i);

  if constexpr (!MIXED) {
    const double2 E = root_E64(f, w, tau, P.d, ms, ns, S);
    if (combined) {
      // conj_s(sum_t c_t A_t) E for each polarization (conj_s: conjugate
      // when s < 0)
      const double2 AP = amp64(a0, tau), AX = amp64(a1, tau);
      const double py = AP.y * P.sd, xy = AX.y * P.sd;
      acc.v[0] += AP.x * E.x - py * E.y;
      acc.v[1] += AP.x * E.y + py * E.x;
      acc.v[2] += AX.x * E.x - xy * E.y;
      acc.v[3] += AX.x * E.y + xy * E.x;
    } else {
      double2 cP = M.cP, cX = M.cX;
      if (M.gm) {
        const GroupMember mb = M.gm[0];
        cP = make_double2(mb.cp_re, neg ? -mb.cp_im : mb.cp_im);
        cX = make_double2(mb.cx_re, neg ? -mb.cx_im : mb.cx_im);
      }
      const double2 A = amp64(a0, tau);
      const double ay = A.y * P.sd;  // A conjugated on s < 0 pieces
      const double Wr = A.x * E.x - ay * E.y, Wi = A.x * E.y + ay * E.x;
      acc.v[0] += cP.x * Wr - cP.y * Wi;
      acc.v[1] += cP.x * Wi + cP.y * Wr;
      acc.v[2] += cX.x * Wr - cX.y * Wi;
      acc.v[3] += cX.x * Wi + cX.y * Wr;
    }
  } else {
    const float2 E = root_E32(f, w, tau, P.d, ms, ns, S);
    const float u = amp_u32(tau, S);
    const float sd = (float)P.sd;
    if (combined) {
      const float2 AP = amp32(a0, u), AX = amp32(a1, u);
      const float py = AP.y * sd, xy = AX.y * sd;
      acc.add(0, AP.x * E.x - py * E.y);
      acc.add(1, AP.x * E.y + py * E.x);
      acc.add(2, AX.x * E.x - xy * E.y);
      acc.add(3, AX.x * E.y + xy * E.x);
    } else {
      float4 c32 = M.c32;
      if (M.gm32) {
        c32 = M.gm32[0].c;
        if (neg) {
          c32.y = -c32.y;
          c32.w = -c32.w;
        }
      }
      const float2 A = amp32(a0, u);
      const float ay = A.y * sd;
      const float Wr = A.x * E.x - ay * E.y, Wi = A.x * E.y + ay * E.x;
      const float pr = c32.x, pi = c32.y, xr = c32.z, xi = c32.w;
      acc.add(0, pr * Wr - pi * Wi);
      acc.add(1, pr * Wi + pi * Wr);
      acc.add(2, xr * Wr - xi * Wi);
      acc.add(3, xr * Wi + xi * Wr);
    }
  }
}

// Cooperative copy of one waveform's shared trajectory tables into LDS
// (caller synchronises).
__device__ __forceinline__ Lds stage_lds(const Prepared& p, double* lds) {
  const int K = p.K, nseg = K - 1;
  KnotRec* kn = (KnotRec*)lds;
  SegCoef* sc = (SegCoef*)(lds + 6 * (size_t)K);
  for (int i = threadIdx.x; i < K; i += blockDim.x) {
    KnotRec r;
    r.Fp = p.Fphi[i];
    r.Fr = p.Fr[i];
    r.t = p.t[i];
    r.Pp = reduce_2pi(p.Phiphi[i]);
    r.Pr = reduce_2pi(p.Phir[i]);
    r.h = (i + 1 < K) ? p.t[i + 1] - p.t[i] : 0.0;
    kn[i] = r;
  }
  for (int i = threadIdx.x; i < nseg; i += blockDim.x) {
    SegCoef c;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      c.cFp[k] = p.tcoef[((size_t)0 * nseg + i) * 4 + 1 + k];
      c.cFr[k] = p.tcoef[((size_t)1 * nseg + i) * 4 + 1 + k];
      c.cPp[k] = p.tcoef[((size_t)2 * nseg + i) * 4 + 1 + k];
      c.cPr[k] = p.tcoef[((size_t)3 * nseg + i) * 4 + 1 + k];
    }
    sc[i] = c;
  }
  return Lds{(const klds KnotRec*)kn, (const klds SegCoef*)sc};
}

// Active-mode list of a block: at most kListCap mode indices at a time, in
// LDS in front of the trajectory tables, followed by the per-wave counts of
// the scan.
constexpr int kListCap = 512;
// Modes examined per lane and round of the active-mode scan.
constexpr int kModesPerLane = 16;
constexpr size_t kHeadDoubles = (kListCap + 8) / 2;

// Bins of one block: WAVES waves, each owning BPL consecutive 64-bin tiles.
template <int BPL, int WAVES>
constexpr int block_bins() {
  return 64 * BPL * WAVES;
}

// Zeros for the bins of a block outside every voice's range.
template <bool MIXED, int BPL, int WAVES>
__device__ __forceinline__ void zero_block(void* hp, void* hc, int Nf, int kb) {
  for (int t = threadIdx.x; t < block_bins<BPL, WAVES>(); t += 64 * WAVES) {
    const int k = kb + t;
    if (k < Nf) {
      if constexpr (MIXED) {
        ((float2*)hp)[k] = make_float2(0.f, 0.f);
        ((float2*)hc)[k] = make_float2(0.f, 0.f);
      } else {
        ((double2*)hp)[k] = make_double2(0.0, 0.0);
        ((double2*)hc)[k] = make_double2(0.0, 0.0);
      }
    }
  }
}

// Writes the active modes of round `base` with list position in
// [c0, c0 + kListCap) (hits: bit j <=> mode wbase + 64 j + lane is active;
// off: list position of the wave's first hit).
__device__ __forceinline__ void write_list(int* list, uint32_t hits, int wbase, int off, int c0) {
  const int lane = threadIdx.x & 63;
  const unsigned long long lanes_below = (1ull << lane) - 1ull;
  int pos = off;
#pragma unroll
  for (int j = 0; j < kModesPerLane; ++j) {
    const unsigned long long bm = __ballot((hits >> j) & 1u);
    if ((hits >> j) & 1u) {
      const int e = pos + __popcll(bm & lanes_below) - c0;
      if (e >= 0 && e < kListCap) list[e] = wbase + j * 64 + lane;
    }
    pos += __popcll(bm);
  }
}

// One wave's pass over list entries [0, n) for its 64-bin tile [ks, ke]:
// every piece of every listed voice group (or, ungrouped, mode) that has bins
// in the tile is evaluated by the lanes whose bin lies in the piece's range,
// in list order and piece order.  A group's pieces, range and mode numbers
// are its first member's.  The mode, range, piece and member tables are
// read-only here and are read through the constant address space, so that
// their wave-uniform records come in by scalar loads.
template <bool MIXED>
__device__ __forceinline__ void walk_list(const Prepared& p, const void* __restrict__ amp, const int* list, int n,
                                          int ks, int ke, double f, double w, const Lds& L, Acc<MIXED>& acc) {
  const int lane = threadIdx.x & 63;
  const int k = ks + lane;
  const int nseg = p.K - 1;
  const bool grouped = p.gmem != nullptr;
  for (int e = 0; e < n; ++e) {
    // a position of the sorted rows (grouped) or a row
    const int j = __builtin_amdgcn_readfirstlane(list[e]);
    Members<MIXED> M;
    M.gm = nullptr;
    M.gm32 = nullptr;
    M.g = 1;
    M.mode = j;
    if (grouped) {
      M.gm = (const kconst GroupMember*)p.gmem + j;
      if constexpr (MIXED) M.gm32 = (const kconst GroupMember32*)p.gmem32 + j;
      M.g = ((const kconst int32_t*)p.gsize)[j];
      M.mode = M.gm[0].mode;
    }
    const int mode = M.mode;
    // the whole 64-B record in one scalar load: its bin range decides, its
    // constants follow (a test on the range table first, with short-circuit
    // evaluation, would cost dependent round trips per entry)
    const ModeConst md = ((const kconst ModeConst*)p.modes)[mode];
    if ((md.k_lo > ke) | (md.k_hi < ks)) continue;
    const kconst Piece* pcs = (const kconst Piece*)p.pieces + (size_t)mode * kMaxPieces;
    for (int q = 0; q < md.npieces; ++q) {
      const Piece P = pcs[q];
      // bins of this piece in the tile (wave-uniform)
      const int ka = max(ks, P.k_lo);
      const int kz = min(ke, P.k_hi);
      if (ka > kz) continue;
      if (k >= ka && k <= kz) {
        const bool neg = P.s < 0;
        const double ms = neg ? -md.m : md.m, ns = neg ? -md.n : md.n;
        if (!grouped) {
          M.cP = make_double2(md.cp_re, neg ? -md.cp_im : md.cp_im);
          M.cX = make_double2(md.cx_re, neg ? -md.cx_im : md.cx_im);
          if constexpr (MIXED) {
            // the FP32 mode constants, wave-uniform (scalar load), conjugated on s < 0
            M.c32 = ((const kconst float4*)p.modes32)[mode];
            if (neg) {
              M.c32.y = -M.c32.y;
              M.c32.w = -M.c32.w;
            }
          }
        }
        eval_bin<MIXED>(f, w, P, ms, ns, neg, M, amp, nseg, L, acc);
      }
    }
  }
}

// Likelihood terms of bin k for the model values hw (h_+ re, im, h_x re, im)
// added to t: wS |d - hw|^2, wS |hw|^2 and wS Re(conj(d) hw), summed over the
// two channels.
template <bool MIXED>
__device__ __forceinline__ void ll_terms(const Sink& o, int k, const double hw[4], double t[3]) {
  double d[4];
  if constexpr (MIXED) {
    const float2 a = ((const float2*)o.d_p)[k], b = ((const float2*)o.d_c)[k];
    d[0] = a.x;
    d[1] = a.y;
    d[2] = b.x;
    d[3] = b.y;
  } else {
    const double2 a = ((const double2*)o.d_p)[k], b = ((const double2*)o.d_c)[k];
    d[0] = a.x;
    d[1] = a.y;
    d[2] = b.x;
    d[3] = b.y;
  }
  double s1 = 0.0, s2 = 0.0, s3 = 0.0;
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    const double e = d[c] - hw[c];
    s1 = __builtin_fma(e, e, s1);
    s2 = __builtin_fma(hw[c], hw[c], s2);
    s3 = __builtin_fma(d[c], hw[c], s3);
  }
  const double ws = o.wS[k];
  t[0] = __builtin_fma(ws, s1, t[0]);
  t[1] = __builtin_fma(ws, s2, t[1]);
  t[2] = __builtin_fma(ws, s3, t[2]);
}

// Hands the sums of one 64-bin tile (global tile index `tile`, this lane's
// bin k) to the sink: stores them, or forms the lane's likelihood terms, sums
// them over the wave (fixed butterfly order) and writes the tile's partials.
// With the Hann kernel, h_w(f_k) = h_k / 2 - (h_{k-1} + h_{k+1}) / 4 takes
// the neighbours from the adjacent lanes; lanes 0 and 63 leave their terms to
// the finishing kernel, which has the neighbouring tiles' edge records.  On
// the mixed path the model is rounded to FP32 first, as the stored waveform
// would be.
template <bool MIXED, bool LL>
__device__ __forceinline__ void emit(const Sink& o, int tile, int k, int Nf, const Acc<MIXED>& acc) {
  if constexpr (!LL) {
    if (k < Nf) {
      if constexpr (MIXED) {
        float v[4];
#pragma unroll
        for (int c = 0; c < 4; ++c) v[c] = (float)acc.v[c];
        ((float2*)o.hp)[k] = make_float2(v[0], v[1]);
        ((float2*)o.hc)[k] = make_float2(v[2], v[3]);
      } else {
        ((double2*)o.hp)[k] = make_double2(acc.v[0], acc.v[1]);
        ((double2*)o.hc)[k] = make_double2(acc.v[2], acc.v[3]);
      }
    }
  } else {
    const int lane = threadIdx.x & 63;
    const bool in = k < Nf;
    double h[4], hw[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) h[c] = in ? (MIXED ? (double)(float)acc.v[c] : (double)acc.v[c]) : 0.0;
    if (o.hann) {
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        const double lft = __shfl_up(h[c], 1, 64), rgt = __shfl_down(h[c], 1, 64);
        hw[c] = 0.5 * h[c] - 0.25 * (lft + rgt);
      }
      if (lane < 2 || lane >= 62) {
        double* e = o.edge + ((size_t)tile * 4 + (lane < 2 ? lane : lane - 60)) * 4;
#pragma unroll
        for (int c = 0; c < 4; ++c) e[c] = h[c];
      }
    } else {
#pragma unroll
      for (int c = 0; c < 4; ++c) hw[c] = h[c];
    }
    double t[3] = {0.0, 0.0, 0.0};
    if (in && !(o.hann && (lane == 0 || lane == 63))) ll_terms<MIXED>(o, k, hw, t);
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
#pragma unroll
      for (int q = 0; q < 3; ++q) t[q] += __shfl_xor(t[q], off, 64);
    }
    if (lane == 0) {
      double* q = o.partial + (size_t)tile * 3;
      q[0] = t[0];
      q[1] = t[1];
      q[2] = t[2];
    }
  }
}

// A block with no bins in any voice's range: zeros (the waveform) or a zero
// model (the likelihood).
template <bool MIXED, int BPL, int WAVES, bool LL>
__device__ __forceinline__ void zero_tiles(const Sink& out, int Nf, int kb) {
  if constexpr (LL) {
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    Acc<MIXED> z;
    z.zero();
#pragma unroll 1
    for (int j = 0; j < BPL; ++j) {
      const int ks = kb + (wave * BPL + j) * 64;
      emit<MIXED, true>(out, ks >> 6, ks + (int)(threadIdx.x & 63), Nf, z);
    }
  } else {
    zero_block<MIXED, BPL, WAVES>(out.hp, out.hc, Nf, kb);
  }
}

// One workgroup's block of WAVES * BPL * 64 contiguous bins starting at kb;
// wave w owns the BPL tiles [kb + 64 (w BPL + j), + 64).
//  1. The workgroup lists the modes whose bin range meets the block: wave w
//     scans a contiguous run of 64 * kModesPerLane modes per round with
//     coalesced loads of the range table, compacts the hits by ballot and
//     writes them, after the hits of lower waves, into an LDS list in
//     increasing mode order.
//  2. Each wave walks the list for each of its tiles; every lane sums all
//     contributions to its bin in one register accumulator, in mode and
//     piece order, and stores the bin.
// The sum of every bin is taken by one lane in a fixed order, so the result
// does not depend on scheduling, on the block shape or on the tile size.
// list: LDS of kListCap + 8 ints.
// stage(): the caller's staging of the waveform's trajectory tables in LDS
// (called by every thread; process_block then synchronises), returning their
// addresses.  eager: stage before the scan of the mode table, so that the two
// latencies overlap other work (the block is known to lie inside the bin
// envelope of the voices); otherwise only once the scan has found voices.
template <bool MIXED, int BPL, int WAVES, bool LL, typename Stage>
__device__ __forceinline__ void process_block(const Prepared& p, const void* __restrict__ amp, const Sink& out,
                                              int kb, int* list, Stage stage, bool eager) {
  constexpr int CHUNK = 64 * kModesPerLane;
  // the wave index is uniform: taken into a scalar register, it makes the
  // tile bounds and every test against them scalar
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
  const int Nf = p.Nf;
  const int kbe = min(kb + block_bins<BPL, WAVES>() - 1, Nf - 1);
  int* wcount = list + kListCap;

  // 1. scan, in rounds of WAVES * CHUNK modes
  const int rounds = (p.Nm + WAVES * CHUNK - 1) / (WAVES * CHUNK);
  bool single = false;  // one round whose hits fit the list: built once, walked for every tile
  int total = 0, off = 0, wbase = 0;
  uint32_t hits = 0;
  auto scan = [&](int base) {
    wbase = base + wave * CHUNK;
    hits = 0;
    const kconst int2* kr = (const kconst int2*)(p.gkr ? p.gkr : p.mode_kr) + wbase + lane;
    const int lim = p.Nm - wbase - lane;
#pragma unroll 4
    for (int j = 0; j < kModesPerLane; ++j) {
      if (j * 64 < lim) {
        const int2 r = kr[j * 64];
        if (r.x <= kbe && r.y >= kb) hits |= 1u << j;
      }
    }
    int cnt = 0;
#pragma unroll
    for (int j = 0; j < kModesPerLane; ++j) cnt += __popcll(__ballot((hits >> j) & 1u));
    __syncthreads();  // the previous list has been consumed
    if (lane == 0) wcount[wave] = cnt;
    __syncthreads();
    off = 0;
    total = 0;
#pragma unroll
    for (int v = 0; v < WAVES; ++v) {
      const int c = wcount[v];
      off += v < wave ? c : 0;
      total += c;
    }
  };
  Lds L;
  if (eager) {
    L = stage();
    __syncthreads();
  }
  if (rounds == 1) {
    scan(0);
    if (total == 0) {
      // no voice has bins here: nothing (more) to stage or evaluate
      zero_tiles<MIXED, BPL, WAVES, LL>(out, Nf, kb);
      return;
    }
    if (!eager) L = stage();
    if (total <= kListCap) {
      single = true;
      write_list(list, hits, wbase, off, 0);
    }
    __syncthreads();  // the tables and the list are in place
  } else if (!eager) {
    L = stage();
    __syncthreads();
  }

  // 2. evaluate, tile by tile
#pragma unroll 1
  for (int j = 0; j < BPL; ++j) {
    const int ks = kb + (wave * BPL + j) * 64;
    const int ke = min(ks + 63, Nf - 1);
    const int k = ks + lane;
    const double f = (k < Nf) ? p.f[k] : 0.0;
    const double w = kTwoPiHi * f;
    Acc<MIXED> acc;
    acc.zero();
    if (single) {
      if (ks <= ke) walk_list<MIXED>(p, amp, list, total, ks, ke, f, w, L, acc);
    } else {
      // many active modes: rebuild the list window by window (every wave
      // takes part in every rebuild)
      for (int r = 0; r < rounds; ++r) {
        scan(r * WAVES * CHUNK);
        for (int c0 = 0; c0 < total; c0 += kListCap) {
          if (c0 > 0) __syncthreads();  // the previous window has been consumed
          write_list(list, hits, wbase, off, c0);
          __syncthreads();
          if (ks <= ke) walk_list<MIXED>(p, amp, list, min(kListCap, total - c0), ks, ke, f, w, L, acc);
        }
      }
    }
    emit<MIXED, LL>(out, ks >> 6, k, Nf, acc);
  }
}

// Occupancy target of the gather kernels, in waves per SIMD (register
// budget 512 / waves VGPRs).  The FP64 evaluation would take more than 128
// VGPRs; bounded to 4 waves (a few spills, outside the evaluation loop) it
// runs faster than at 3 without spills, and at 5 no faster.  The mixed one
// fits 5 waves (96 VGPRs, spills outside the evaluation loop), which is
// faster than 4 in the single-waveform and the batch kernel.
template <bool MIXED>
constexpr int gather_min_waves() {
  return MIXED ? 5 : 4;
}

template <bool MIXED>
constexpr int gather_batch_min_waves() {
  return MIXED ? 5 : 4;
}

// LL = false: the waveform; LL = true: the likelihood partials (Sink).
template <bool MIXED, int BPL, int WAVES, bool LL>
__global__ __launch_bounds__(64 * WAVES, gather_min_waves<MIXED>()) void gather_kernel(GatherArgs a) {
  extern __shared__ __align__(16) double lds[];
  const Prepared& p = a.p;
  const int kb = (int)blockIdx.x * block_bins<BPL, WAVES>();
  // a waveform whose inputs failed the checks has a zero model, and so do
  // the blocks outside the bin envelope of its voices (after a fused set-up:
  // the check workgroups' slots, every wave reading all of them, and no
  // envelope)
  bool bad;
  int env_lo = 0, env_hi = INT_MAX;
  if (p.nslots > 0) {
    int v = 0;
    for (int j = (int)(threadIdx.x & 63); j < p.nslots; j += 64) v |= p.slots[j];
    bad = __any(v != 0);
  } else {
    const kconst int32_t* st = (const kconst int32_t*)p.status;
    bad = st[0] != 0;
    env_lo = st[1];
    env_hi = st[2];
  }
  if (bad || kb + block_bins<BPL, WAVES>() - 1 < env_lo || kb > env_hi) {
    zero_tiles<MIXED, BPL, WAVES, LL>(a.out, p.Nf, kb);
    return;
  }
  int* list = (int*)lds;
  // a formed envelope (large mode tables) means the block most likely has
  // voices: stage the tables at once
  const bool eager = env_lo > 0 || env_hi < INT_MAX;
  process_block<MIXED, BPL, WAVES, LL>(p, a.amp, a.out, kb, list, [&]() { return stage_lds(p, lds + kHeadDoubles); },
                                      eager);
}

// Completes the likelihood of one waveform from the gather's per-tile
// partials, in two fixed-order stages.  Stage 1, one thread per tile: the
// tile's partials and, with the Hann kernel, the terms of its first and last
// bin, whose neighbours come from the edge records of the tile and of the
// tiles beside it (outside the grid the model is zero; below the first bin of
// the grid h(-f_1) = conj h(f_1), the transform of a real series); then a
// tree over the workgroup, one triple per workgroup in block_sums.  Stage 2
// (one workgroup) adds the workgroups' triples in order:
// out = (-1/2 sum wS |d - h_w|^2, sum wS |h_w|^2, sum wS Re(conj(d) h_w)).
constexpr int kLLThreads = 256;

// One workgroup of stage 1: the triple of tiles [x kLLThreads, (x + 1)
// kLLThreads) of one waveform into dst[3].
template <bool MIXED>
__device__ __forceinline__ void loglike_tile_block(const Sink& o, int Nf, int x, double* dst) {
  __shared__ double red[3][kLLThreads];
  const int ntiles = (Nf + 63) / 64;
  const int i = x * kLLThreads + (int)threadIdx.x;
  double t[3] = {0.0, 0.0, 0.0};
  if (i < ntiles) {
#pragma unroll
    for (int q = 0; q < 3; ++q) t[q] = o.partial[(size_t)i * 3 + q];
    if (o.hann) {
      const double* e = o.edge + (size_t)i * 16;  // lanes 0, 1, 62, 63 of tile i
      double hw[4];
      const int k0 = 64 * i;
      const double* prv = o.edge + (size_t)(i > 0 ? i - 1 : 0) * 16 + 12;  // lane 63 of tile i - 1
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        const double hm = (i > 0) ? prv[c] : ((c & 1) ? -e[4 + c] : e[4 + c]);
        hw[c] = 0.5 * e[c] - 0.25 * (hm + e[4 + c]);
      }
      ll_terms<MIXED>(o, k0, hw, t);
      const int k1 = 64 * i + 63;
      if (k1 < Nf) {
        const double* nxt = o.edge + (size_t)(i + 1 < ntiles ? i + 1 : i) * 16;  // lane 0 of tile i + 1
#pragma unroll
        for (int c = 0; c < 4; ++c) {
          const double hp1 = (i + 1 < ntiles) ? nxt[c] : 0.0;
          hw[c] = 0.5 * e[12 + c] - 0.25 * (e[8 + c] + hp1);
        }
        ll_terms<MIXED>(o, k1, hw, t);
      }
    }
  }
#pragma unroll
  for (int q = 0; q < 3; ++q) red[q][threadIdx.x] = t[q];
  __syncthreads();
  for (int w = kLLThreads / 2; w >= 1; w >>= 1) {
    if ((int)threadIdx.x < w) {
#pragma unroll
      for (int q = 0; q < 3; ++q) red[q][threadIdx.x] += red[q][threadIdx.x + w];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
#pragma unroll
    for (int q = 0; q < 3; ++q) dst[q] = red[q][0];
  }
}

template <bool MIXED>
__global__ __launch_bounds__(kLLThreads) void loglike_tiles_kernel(Sink o, int Nf, double* block_sums) {
  loglike_tile_block<MIXED>(o, Nf, (int)blockIdx.x, block_sums + (size_t)blockIdx.x * 3);
}

// Stage 1 for a batch: blockIdx.y selects the waveform; its workgroups past
// the waveform's own count leave zeros (stage 2 then adds the same terms in
// the same order as for a single waveform).
template <bool MIXED>
__global__ __launch_bounds__(kLLThreads) void loglike_tiles_batch_kernel(const WaveItem* __restrict__ items, int hann,
                                                                         int nbmax, double* block_sums) {
  const WaveItem w = ((const kconst WaveItem*)items)[blockIdx.y];
  Sink o{};
  o.d_p = w.d_p;
  o.d_c = w.d_c;
  o.wS = w.wS;
  o.partial = w.ll_partial;
  o.edge = w.ll_edge;
  o.hann = hann;
  loglike_tile_block<MIXED>(o, w.Nf, (int)blockIdx.x, block_sums + ((size_t)blockIdx.y * nbmax + blockIdx.x) * 3);
}

// Stage 2; workgroup b adds the nblocks triples of waveform b into out[b].
__global__ __launch_bounds__(kLLThreads) void loglike_total_kernel(const double* block_sums, int nblocks,
                                                                   double* out) {
  __shared__ double red[3][kLLThreads];
  block_sums += (size_t)blockIdx.x * nblocks * 3;
  out += (size_t)blockIdx.x * 3;
  double t[3] = {0.0, 0.0, 0.0};
  for (int b = threadIdx.x; b < nblocks; b += kLLThreads) {
#pragma unroll
    for (int q = 0; q < 3; ++q) t[q] += block_sums[(size_t)b * 3 + q];
  }
#pragma unroll
  for (int q = 0; q < 3; ++q) red[q][threadIdx.x] = t[q];
  __syncthreads();
  for (int w = kLLThreads / 2; w >= 1; w >>= 1) {
    if ((int)threadIdx.x < w) {
#pragma unroll
      for (int q = 0; q < 3; ++q) red[q][threadIdx.x] += red[q][threadIdx.x + w];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    out[0] = -0.5 * red[0][0];
    out[1] = red[1][0];
    out[2] = red[2][0];
  }
}

// Persistent gather over a batch: every workgroup repeatedly takes the next
// block (waveform b, bins [j B, (j + 1) B) with B = 64 BPL WAVES) from a
// device counter and evaluates it exactly as the single-waveform kernel
// would, restaging the LDS tables when the waveform changes.  The counter
// only schedules; every output element is computed in a fixed order, so
// results do not depend on the schedule.  Every workgroup leaves the loop
// once the counter passes the last block.
template <bool MIXED, int BPL, int WAVES, bool LL>
__global__ __launch_bounds__(64 * WAVES, gather_batch_min_waves<MIXED>()) void gather_batch_kernel(const WaveItem* __restrict__ items, int B,
                                                                const int32_t* __restrict__ item_prefix,
                                                                int total_items, int* __restrict__ counter,
                                                                int hann) {
  extern __shared__ __align__(16) double lds[];
  __shared__ int s_item;
  int* list = (int*)lds;
  double* tables = lds + kHeadDoubles;
  int cached = -1;
  Lds L{};
  for (;;) {
    __syncthreads();
    if (threadIdx.x == 0) s_item = atomicAdd(counter, 1);
    __syncthreads();
    const int it = s_item;
    if (it >= total_items) break;
    // the records are read-only here (constant address space: scalar loads)
    const kconst int32_t* pre = (const kconst int32_t*)item_prefix;
    int lo = 0, hi = B - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (pre[mid] <= it)
        lo = mid;
      else
        hi = mid - 1;
    }
    const WaveItem w = ((const kconst WaveItem*)items)[lo];
    const Prepared p = prepared_of(w);
    const int kb = (it - pre[lo]) * block_bins<BPL, WAVES>();
    Sink out{};
    out.hp = w.hp;
    out.hc = w.hc;
    if constexpr (LL) {
      out.d_p = w.d_p;
      out.d_c = w.d_c;
      out.wS = w.wS;
      out.partial = w.ll_partial;
      out.edge = w.ll_edge;
      out.hann = hann;
    }
    const kconst int32_t* st = (const kconst int32_t*)p.status;
    if (st[0] != 0 || kb + block_bins<BPL, WAVES>() - 1 < st[1] || kb > st[2]) {
      zero_tiles<MIXED, BPL, WAVES, LL>(out, p.Nf, kb);
      continue;
    }
    // the tables are restaged only when the waveform changes
    process_block<MIXED, BPL, WAVES, LL>(p, MIXED ? (const void*)w.acoef32 : (const void*)w.acoef, out, kb, list,
                                        [&]() {
                                          if (lo != cached) {
                                            L = stage_lds(p, tables);
                                            cached = lo;
                                          }
                                          return L;
                                        },
                                        true);
  }
}

__global__ void reset_counter_kernel(int* counter) { *counter = 0; }

// FP32 normalised amplitude coefficients for the mixed path when the caller
// gives the FP64 coefficients (FDEMRI_COEFFS_GIVEN) (amp32_segment); splined
// amplitudes get them from the spline kernels, with the same arithmetic.

__global__ void amp32_kernel(int Nm, int K, const double* __restrict__ t, const double* __restrict__ acoef,
                             float* __restrict__ acoef32) {
  const int nseg = K - 1;
  const long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (long)Nm * nseg) return;
  const int i = (int)(idx % nseg);
  amp32_segment(acoef + idx * 8, t[i + 1] - t[i], acoef32 + idx * 8);
}

// Batched: one thread per (waveform, mode, segment) through the prefix of
// Nm_b (K_b - 1); members without given coefficients have theirs already.
__global__ void amp32_batch_kernel(const WaveItem* __restrict__ items, int B, const int32_t* __restrict__ amp_prefix,
                                   int total) {
  const int g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= total) return;
  int lo = 0, hi = B - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (amp_prefix[mid] <= g)
      lo = mid;
    else
      hi = mid - 1;
  }
  const WaveItem& w = items[lo];
  if (!(w.flags & FDEMRI_COEFFS_GIVEN)) return;
  const int idx = g - amp_prefix[lo];
  const int i = idx % (w.K - 1);
  amp32_segment(w.acoef + (size_t)idx * 8, w.t[i + 1] - w.t[i], w.acoef32 + (size_t)idx * 8);
}

hipError_t launch_amp32(int Nm, int K, const double* t, const double* acoef, float* acoef32, hipStream_t stream) {
  const long total = (long)Nm * (K - 1);
  const int threads = 256;
  amp32_kernel<<<dim3((unsigned)((total + threads - 1) / threads)), threads, 0, stream>>>(Nm, K, t, acoef, acoef32);
  return hipGetLastError();
}

hipError_t launch_amp32_batch(const WaveItem* items, int B, const int32_t* amp_prefix, int total, hipStream_t stream) {
  const int threads = 256;
  amp32_batch_kernel<<<(total + threads - 1) / threads, threads, 0, stream>>>(items, B, amp_prefix, total);
  return hipGetLastError();
}

size_t gather_lds_bytes(int K) { return (size_t)K * sizeof(KnotRec) + (size_t)(K - 1) * sizeof(SegCoef); }

template <bool MIXED, int BPL, int WAVES, bool LL>
static hipError_t launch_gather_t(const GatherArgs& a, hipStream_t stream) {
  constexpr int per_block = block_bins<BPL, WAVES>();
  const long blocks = ((long)a.p.Nf + per_block - 1) / per_block;
  const size_t red = kHeadDoubles * sizeof(double);
  const size_t lds = gather_lds_bytes(a.p.K) + red;
  static bool attr_set = false;
  if (!attr_set) {
    (void)hipFuncSetAttribute((const void*)gather_kernel<MIXED, BPL, WAVES, LL>,
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)(gather_lds_bytes(kMaxKnots) + red));
    attr_set = true;
  }
  gather_kernel<MIXED, BPL, WAVES, LL><<<dim3((unsigned)blocks), dim3(64 * WAVES), lds, stream>>>(a);
  return hipGetLastError();
}

template <bool LL>
static hipError_t launch_gather(const GatherArgs& a, bool mixed, int bpl, hipStream_t stream) {
  if (mixed) {
    if (bpl == 1) return launch_gather_t<true, 1, 4, LL>(a, stream);
    if (bpl == 2) return launch_gather_t<true, 2, 4, LL>(a, stream);
    return launch_gather_t<true, 4, 4, LL>(a, stream);
  }
  if (bpl == 1) return launch_gather_t<false, 1, 4, LL>(a, stream);
  if (bpl == 2) return launch_gather_t<false, 2, 4, LL>(a, stream);
  return launch_gather_t<false, 4, 4, LL>(a, stream);
}

hipError_t launch_gather_flat(const Prepared& p, const float* acoef32, void* hp, void* hc, bool mixed, int bpl,
                              hipStream_t stream) {
  GatherArgs a{};
  a.p = p;
  a.amp = mixed ? (const void*)acoef32 : (const void*)p.acoef;
  a.out.hp = hp;
  a.out.hc = hc;
  return launch_gather<false>(a, mixed, bpl, stream);
}

// Tiles of the gather grid for Nf bins (every tile of every block, also those
// past the last bin): the size of the likelihood partial and edge arrays; the
// workgroup triples of the first reduction stage follow the partials.
int loglike_tiles(int Nf, int bpl) {
  const int per_block = 64 * bpl * 4;
  return (Nf + per_block - 1) / per_block * bpl * 4;
}

static int loglike_reduce_blocks(int Nf) { return ((Nf + 63) / 64 + kLLThreads - 1) / kLLThreads; }

// Doubles of likelihood scratch before the edge records: partials, then the
// triples of the first reduction stage.
size_t loglike_partial_doubles(int Nf, int bpl) {
  return (size_t)loglike_tiles(Nf, bpl) * 3 + (size_t)loglike_reduce_blocks(Nf) * 3;
}

hipError_t launch_loglike(const Prepared& p, const float* acoef32, bool mixed, int bpl, const void* d_p,
                          const void* d_c, const double* wS, int hann, double* partial, double* edge, double* out,
                          hipStream_t stream) {
  GatherArgs a{};
  a.p = p;
  a.amp = mixed ? (const void*)acoef32 : (const void*)p.acoef;
  a.out.d_p = d_p;
  a.out.d_c = d_c;
  a.out.wS = wS;
  a.out.partial = partial;
  a.out.edge = edge;
  a.out.hann = hann;
  hipError_t e = launch_gather<true>(a, mixed, bpl, stream);
  if (e != hipSuccess) return e;
  const int nb = loglike_reduce_blocks(p.Nf);
  double* block_sums = partial + (size_t)loglike_tiles(p.Nf, bpl) * 3;
  if (mixed)
    loglike_tiles_kernel<true><<<nb, kLLThreads, 0, stream>>>(a.out, p.Nf, block_sums);
  else
    loglike_tiles_kernel<false><<<nb, kLLThreads, 0, stream>>>(a.out, p.Nf, block_sums);
  loglike_total_kernel<<<1, kLLThreads, 0, stream>>>(block_sums, nb, out);
  return hipGetLastError();
}

template <bool MIXED, int BPL, int WAVES, bool LL>
static hipError_t launch_gather_batch_t(const WaveItem* items, int B, const int32_t* item_prefix, int total_items,
                                        int* counter, int Kmax, int grid, int hann, hipStream_t stream) {
  const size_t red = kHeadDoubles * sizeof(double);
  const size_t lds = gather_lds_bytes(Kmax) + red;
  static bool attr_set = false;
  if (!attr_set) {
    (void)hipFuncSetAttribute((const void*)gather_batch_kernel<MIXED, BPL, WAVES, LL>,
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)(gather_lds_bytes(kMaxKnots) + red));
    attr_set = true;
  }
  reset_counter_kernel<<<1, 1, 0, stream>>>(counter);
  gather_batch_kernel<MIXED, BPL, WAVES, LL><<<dim3(grid), dim3(64 * WAVES), lds, stream>>>(
      items, B, item_prefix, total_items, counter, hann);
  return hipGetLastError();
}

// Number of workgroups of the persistent kernel: enough to fill every CU.
template <bool MIXED, int BPL, int WAVES, bool LL>
static int persistent_grid(int Kmax) {
  int dev = 0, ncu = 0, per_cu = 0;
  (void)hipGetDevice(&dev);
  (void)hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
  (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void*)gather_batch_kernel<MIXED, BPL, WAVES, LL>,
                                                     64 * WAVES,
                                                     gather_lds_bytes(Kmax) + kHeadDoubles * sizeof(double));
  if (ncu <= 0) ncu = 256;
  if (per_cu <= 0) per_cu = 1;
  return ncu * per_cu;
}

int gather_items_per_waveform(int Nf, int bpl) {
  const int per_block = 64 * bpl * 4;  // WAVES = 4 in every launch below
  return (Nf + per_block - 1) / per_block;
}

template <bool MIXED, bool LL>
static hipError_t launch_gather_batch_p(const WaveItem* items, int B, const int32_t* item_prefix, int total_items,
                                        int* counter, int Kmax, int bpl, int hann, hipStream_t stream) {
  if (bpl == 1)
    return launch_gather_batch_t<MIXED, 1, 4, LL>(items, B, item_prefix, total_items, counter, Kmax,
                                                  persistent_grid<MIXED, 1, 4, LL>(Kmax), hann, stream);
  if (bpl == 2)
    return launch_gather_batch_t<MIXED, 2, 4, LL>(items, B, item_prefix, total_items, counter, Kmax,
                                                  persistent_grid<MIXED, 2, 4, LL>(Kmax), hann, stream);
  return launch_gather_batch_t<MIXED, 4, 4, LL>(items, B, item_prefix, total_items, counter, Kmax,
                                                persistent_grid<MIXED, 4, 4, LL>(Kmax), hann, stream);
}

hipError_t launch_gather_batch(const WaveItem* items, int B, const int32_t* item_prefix, int total_items,
                               int* counter, int Kmax, bool mixed, int bpl, hipStream_t stream) {
  if (mixed) return launch_gather_batch_p<true, false>(items, B, item_prefix, total_items, counter, Kmax, bpl, 0, stream);
  return launch_gather_batch_p<false, false>(items, B, item_prefix, total_items, counter, Kmax, bpl, 0, stream);
}

// Likelihood stage-1 workgroups of the largest waveform of a batch.
int loglike_batch_reduce_blocks(int Nf_max) { return loglike_reduce_blocks(Nf_max); }

// The fused likelihood of a batch: persistent gather into every waveform's
// partials, then the two reduction stages, out[b][3] per waveform (same
// arithmetic and order as a single-waveform call).  block_sums: B x nbmax x 3.
hipError_t launch_loglike_batch(const WaveItem* items, int B, const int32_t* item_prefix, int total_items,
                                int* counter, int Kmax, bool mixed, int bpl, int hann, int Nf_max,
                                double* block_sums, double* out, hipStream_t stream) {
  hipError_t e = mixed
                     ? launch_gather_batch_p<true, true>(items, B, item_prefix, total_items, counter, Kmax, bpl, hann, stream)
                     : launch_gather_batch_p<false, true>(items, B, item_prefix, total_items, counter, Kmax, bpl, hann,
                                                         stream);
  if (e != hipSuccess) return e;
  const int nbmax = loglike_reduce_blocks(Nf_max);
  const dim3 grid((unsigned)nbmax, (unsigned)B);
  if (mixed)
    loglike_tiles_batch_kernel<true><<<grid, kLLThreads, 0, stream>>>(items, hann, nbmax, block_sums);
  else
    loglike_tiles_batch_kernel<false><<<grid, kLLThreads, 0, stream>>>(items, hann, nbmax, block_sums);
  loglike_total_kernel<<<B, kLLThreads, 0, stream>>>(block_sums, nbmax, out);
  return hipGetLastError();
}

}  // namespace fdemri
