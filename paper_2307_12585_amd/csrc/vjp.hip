// Adjoint of the frequency-domain mode sum: the gradient of a real loss L
// of h_+(f), h_x(f) (e.g. the Whittle log-likelihood of Eq. likelihood) with
// respect to the amplitude and phase spline coefficients, the viewing angles,
// the distance scale and the initial phases, given the cotangents
// g = dL/dRe h + i dL/dIm h.
//
// Per root (fused partner form, E = e^{i psi} G, A the amplitude spline):
//   h_+ += (A c_+)^(s) E,  h_x += (A c_x)^(s) E   ((.)^(s): conjugate when s < 0)
//   dL/da_k    = tau^k [g_+ conj(c_+) + g_x conj(c_x)] conj(E)     (s > 0)
//              = tau^k conj(g_+ c_+ + g_x c_x) E                   (s < 0)
//   dL/dc^phi_k = s m tau^k Im Z, dL/dc^r_k = s n tau^k Im Z,
//              Z = conj(g_+)(A c_+)^(s) E + conj(g_x)(A c_x)^(s) E
//              (psi depends on -s (m Phi_phi + n Phi_r))
//   dL = Re(U_+ dc_+) + Re(U_x dc_x),
//   U_+ = sum conj(g_+) A E (s > 0) + g_+ A conj(E) (s < 0), likewise U_x,
// and c_+, c_x depend on theta, phi and the scale (d/dphi c = i m c).
//
// The forward terms are recomputed, not stored: the bins whose root lies in
// segment i of a voice group (the same segment assignment, bracket and
// arithmetic as the forward gather) are cut into chunks of equal size, each
// wavefront re-evaluates the roots of the chunks it takes and reduces
// moments of conj(g) E in registers, and every row's terms follow from the
// moments summed per (group, segment).  Which wave takes which chunk varies
// from run to run, but every sum runs in a fixed order (a chunk's bins, a
// unit's chunks, the reductions after), so the gradient is deterministic;
// the only atomics count bins and hand out chunks.
#include "evalcore.hpp"
#include "harmonics.hpp"
#include "search.hpp"

#include <rocprim/device/device_scan.hpp>
#include <rocprim/iterator/counting_iterator.hpp>
#include <rocprim/iterator/transform_iterator.hpp>

namespace fdemri {

struct VjpArgs {
  Prepared p;
  const float* acoef32;
  const void* g_hp;
  const void* g_hc;
  double* gA;     // [Nm][nseg][8] coefficient gradient (re, im per power)
  double* PZ;     // [Nm][nseg][4]  sum s tau^k Im Z
  double* Upart;  // [Nm][nseg][4]  partial U_+ (re, im), U_x (re, im)
};

// Sum over the wave of 16 per-lane values by halving exchanges: at each of the
// lane offsets 32, 16, 8 and 4 a lane keeps the half of its values selected
// by that lane bit and adds the partner's copy of the same half, so that lane
// L ends with a partial of value (L >> 2) over 16 lanes; two butterfly steps
// complete it.  Returns in every lane the total of value L >> 2 (fixed order:
// deterministic).  About a third of the exchanges of 16 full butterflies.
__device__ __forceinline__ double wave_sum16(const double v[16]) {
  const int lane = threadIdx.x & 63;
  double a8[8], a4[4], a2[2];
  {
    const bool hi = (lane & 32) != 0;
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const double keep = hi ? v[j + 8] : v[j], send = hi ? v[j] : v[j + 8];
      a8[j] = keep + __shfl_xor(send, 32, 64);
    }
  }
  {
    const bool hi = (lane & 16) != 0;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const double keep = hi ? a8[j + 4] : a8[j], send = hi ? a8[j] : a8[j + 4];
      a4[j] = keep + __shfl_xor(send, 16, 64);
    }
  }
  {
    const bool hi = (lane & 8) != 0;
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const double keep = hi ? a4[j + 2] : a4[j], send = hi ? a4[j] : a4[j + 2];
      a2[j] = keep + __shfl_xor(send, 8, 64);
    }
  }
  const bool hi = (lane & 4) != 0;
  double a1 = (hi ? a2[1] : a2[0]) + __shfl_xor(hi ? a2[0] : a2[1], 4, 64);
  a1 += __shfl_xor(a1, 2, 64);
  a1 += __shfl_xor(a1, 1, 64);
  return a1;
}

// The adjoint's work is split by bins, not by unit: a unit (voice group at
// sorted position j, spline segment i; every row its own group when the
// table is not grouped) owns the bins whose root the forward search places
// in segment i of one of its pieces, and their count varies by orders of
// magnitude (a fast chirp's last segments hold most bins).  The plan kernel
// finds each unit's bin range per piece, the scan gives each unit a run of
// fixed-size chunks of its (piece-concatenated) bins and a map records each
// chunk's unit, the chunk kernel hands the chunks out to the waves through a
// counter, and the finish kernel sums
// each unit's chunks in chunk order and forms every row's terms.
//
// The rows of a group share the pieces, roots and E, so a chunk forms, per
// piece, the moments
//   Mp_k = sum over bins of u^k conj(g_+) E,  Mx_k = sum u^k conj(g_x) E,
// u = tau / h, k = 0..6, and stores them sign-folded,
//   Qp_k = conj(Mp_k) (s > 0), Mp_k (s < 0),  Qx_k likewise,
// so that they add across pieces and chunks and every row's terms follow
// from the sums (a the row's amplitude coefficients in u, a^_j = a_j h^j,
// c its factors):
//   dL/da_k = h^k (conj(c_+) Qp_k + conj(c_x) Qx_k),
//   U_+ = sum_j a^_j conj(Qp_j),  U_x = sum_j a^_j conj(Qx_j)   (k, j = 0..3),
// and the group's sum s tau^k Im Z, Z = conj(g_+) Cp(u)^(s) E + conj(g_x)
// Cx(u)^(s) E with Cp(u) = sum_j Cp_j u^j = sum_t c_+,t A_t(u) (Cx likewise)
// the group's combined amplitude, is
//   s sum u^k Im Z = -h^k sum_j Im(conj(Cp_j) Qp_{j+k} + conj(Cx_j) Qx_{j+k}).  Outputs per row
// of the group: gA (8), Upart (4) and PZ (4; the group's sum at its first
// row, zero at the others, since the phase gradient sums m PZ over the rows).

// bins per chunk: at least kVjpMinChunkIters passes of the wave, and so many
// that the chunks number at most the units plus kVjpChunkCap
constexpr int kVjpMinChunkIters = 32;
constexpr long long kVjpChunkCap = 1 << 19;
constexpr int kVjpMom = 28;  // doubles per chunk: Qp_0..6 (14), Qx_0..6 (14)

__device__ __forceinline__ int vjp_chunk_bins(unsigned long long bins) {
  const unsigned long long per = (bins + 64ull * kVjpChunkCap - 1) / (64ull * kVjpChunkCap);
  return 64 * (int)max(per, (unsigned long long)kVjpMinChunkIters);
}
__device__ __forceinline__ int vjp_chunks(int nb, int ch) { return (nb + ch - 1) / ch; }

struct VjpPlan {
  int2* rng;                 // [Nm * nseg][kMaxPieces] bin range of each piece in the unit (empty: x > y)
  int32_t* nb;               // [Nm * nseg] bins of the unit over its pieces (0: no work, not a group's unit)
  int32_t* off;              // [Nm * nseg] first chunk of the unit (exclusive scan of the chunk counts)
  unsigned long long* ctl;   // [0] bins of all units, [1] the next chunk to hand out
  int32_t* unit_of;          // [chunks] the unit of each chunk
  double* mom;               // [chunks][kVjpMom]
};

struct VjpChunkCount {
  const int32_t* nb;
  const unsigned long long* ctl;
  __device__ int operator()(int u) const { return vjp_chunks(nb[u], vjp_chunk_bins(ctl[0])); }
};

__global__ void vjp_plan_zero_kernel(unsigned long long* ctl) {
  ctl[0] = 0;
  ctl[1] = 0;
}

// One thread per (row, segment) unit: the bins of each piece whose root the
// forward search places in segment i (the largest segment j in
// [seg_a, seg_b] with j == seg_a or d g_j < d f).
__global__ __launch_bounds__(256) void vjp_plan_kernel(Prepared p, VjpPlan v) {
  const int nseg = p.K - 1;
  const long U = (long)p.Nm * nseg;
  const long u = (long)blockIdx.x * blockDim.x + threadIdx.x;
  long long total = 0;
  if (u < U) {
    const int j = (int)(u / nseg), i = (int)(u % nseg);
    const bool grouped = p.gsize != nullptr;
    const int g = grouped ? p.gsize[j] : 1;
    // a waveform whose inputs failed the checks has a zero gradient; a
    // group's other rows are covered by its unit
    if (g > 0 && *p.status == 0) {
      const int lead = grouped ? p.gmem[j].mode : j;
      const ModeConst md = p.modes[lead];
      const double F0 = knot_freq(md.m, p.Fphi[i], md.n, p.Fr[i]);
      const double F1 = knot_freq(md.m, p.Fphi[i + 1], md.n, p.Fr[i + 1]);
      for (int q = 0; q < md.npieces; ++q) {
        const Piece P = p.pieces[(size_t)lead * kMaxPieces + q];
        int kA = P.k_lo, kB = P.k_hi;
        if (i >= P.seg_a && i <= P.seg_b && P.k_lo <= P.k_hi) {
          const double gi = P.s < 0 ? -F0 : F0, gi1 = P.s < 0 ? -F1 : F1;
          if (P.d > 0) {
            if (i > P.seg_a) kA = max(kA, first_gt(p.f, p.Nf, gi));
            if (i < P.seg_b) kB = min(kB, first_gt(p.f, p.Nf, gi1) - 1);
          } else {
            if (i > P.seg_a) kB = min(kB, first_ge(p.f, p.Nf, gi) - 1);
            if (i < P.seg_b) kA = max(kA, first_ge(p.f, p.Nf, gi1));
          }
        } else {
          kA = 1;
          kB = 0;
        }
        if (kA > kB) {
          kA = 1;
          kB = 0;
        }
        v.rng[u * kMaxPieces + q] = make_int2(kA, kB);
        total += kB - kA + 1;
      }
    }
    v.nb[u] = (int32_t)total;
  }
  // the wave's bins, added once
  for (int o = 32; o > 0; o >>= 1) total += __shfl_xor(total, o, 64);
  if ((threadIdx.x & 63) == 0 && total) atomicAdd(&v.ctl[0], (unsigned long long)total);
}

// One thread per unit: its chunks' entries of the chunk-to-unit map.
__global__ __launch_bounds__(256) void vjp_map_kernel(int U, VjpPlan v) {
  const int u = blockIdx.x * blockDim.x + threadIdx.x;
  if (u >= U) return;
  const int nc = vjp_chunks(v.nb[u], vjp_chunk_bins(v.ctl[0]));
  const int o = v.off[u];
  for (int k = 0; k < nc; ++k) v.unit_of[o + k] = u;
}

// Occupancy target in waves per SIMD: the mixed adjoint fits 4; the FP64 one
// would spill inside the bin loop and stays at 3.
template <bool MIXED>
constexpr int vjp_min_waves() {
  return MIXED ? 4 : 3;
}

// Chunks handed out one per wave through the counter until all are taken;
// each writes its sign-folded moments (kVjpMom doubles).
template <bool MIXED>
__global__ __launch_bounds__(256, vjp_min_waves<MIXED>()) void vjp_chunk_kernel(VjpArgs a, VjpPlan v) {
  const Prepared& p = a.p;
  const int nseg = p.K - 1;
  const int U = p.Nm * nseg;
  const int lane = threadIdx.x & 63;
  const int ch = vjp_chunk_bins(*(const kconst unsigned long long*)v.ctl);
  const kconst int32_t* koff = (const kconst int32_t*)v.off;
  const int T = koff[U - 1] + vjp_chunks(((const kconst int32_t*)v.nb)[U - 1], ch);
  const bool grouped = p.gsize != nullptr;
  const kconst double* kt = (const kconst double*)p.t;
  const kconst double* kFp = (const kconst double*)p.Fphi;
  const kconst double* kFr = (const kconst double*)p.Fr;
  for (;;) {
    int c0 = 0;
    if (lane == 0) c0 = (int)atomicAdd(&v.ctl[1], 1ull);
    const int c = __builtin_amdgcn_readfirstlane(__shfl(c0, 0, 64));
    if (c >= T) break;
    const int u = ((const kconst int32_t*)v.unit_of)[c];
    const int b0 = (c - koff[u]) * ch, b1 = b0 + ch;  // the chunk in the unit's concatenated bins
    const int j = u / nseg, i = u % nseg;
    const int g = grouped ? ((const kconst int32_t*)p.gsize)[j] : 1;
    const kconst GroupMember* gm = grouped ? (const kconst GroupMember*)p.gmem + j : nullptr;
    const int lead = grouped ? gm[0].mode : j;
    const ModeConst md = ((const kconst ModeConst*)p.modes)[lead];
    const double m = md.m, n = md.n;
    const double ti = kt[i], h = kt[i + 1] - ti;
    const double F0 = knot_freq(m, kFp[i], n, kFr[i]);
    const double F1 = knot_freq(m, kFp[i + 1], n, kFr[i + 1]);
    const kconst double* cFp = (const kconst double*)p.tcoef + ((size_t)0 * nseg + i) * 4;
    const kconst double* cFr = (const kconst double*)p.tcoef + ((size_t)1 * nseg + i) * 4;
    const kconst double* cPp = (const kconst double*)p.tcoef + ((size_t)2 * nseg + i) * 4;
    const kconst double* cPr = (const kconst double*)p.tcoef + ((size_t)3 * nseg + i) * 4;
    const double Ppr = reduce_2pi(((const kconst double*)p.Phiphi)[i]);
    const double Prr = reduce_2pi(((const kconst double*)p.Phir)[i]);

    // moments, sign-folded per piece as they are added: acc[2k], acc[2k+1] =
    // Qp_k; acc[14 + 2k], acc[15 + 2k] = Qx_k
    double acc[kVjpMom];
#pragma unroll
    for (int r = 0; r < kVjpMom; ++r) acc[r] = 0.0;
    int pos = 0;  // the piece's first bin in the unit's concatenated bins
    for (int q = 0; q < md.npieces && pos < b1; ++q) {
      const int2 rq = ((const kconst int2*)v.rng)[(size_t)u * kMaxPieces + q];
      const int nq = rq.y - rq.x + 1;
      const int lo_b = max(b0, pos), hi_b = min(b1, pos + nq);
      const int kA = rq.x + (lo_b - pos), kB = rq.x + (hi_b - pos) - 1;
      pos += max(nq, 0);
      if (nq <= 0 || kA > kB) continue;
      const Piece P = ((const kconst Piece*)p.pieces)[(size_t)lead * kMaxPieces + q];
      const int s = P.s, d = P.d;
      const double dd_ = (double)d;
      // |F_V| and s Phi_V of this piece on segment i (sign folded into the mode numbers)
      const double ms = s < 0 ? -m : m, ns = s < 0 ? -n : n;
      SegData S;
      S.ti = ti;
      S.h = h;
      S.G0 = s < 0 ? -F0 : F0;
      S.G1 = s < 0 ? -F1 : F1;
      S.q1 = wsum(ms, cFp[1], ns, cFr[1]);
      S.q2 = wsum(ms, cFp[2], ns, cFr[2]);
      S.q3 = wsum(ms, cFp[3], ns, cFr[3]);
      S.r1 = wsum(ms, cPp[1], ns, cPr[1]);
      S.r2 = wsum(ms, cPp[2], ns, cPr[2]);
      S.r3 = wsum(ms, cPp[3], ns, cPr[3]);
      S.Ppi = Ppr;
      S.Pri = Prr;
      // the bracket of the roots in segment i (the piece's end values at its
      // first and last segment); i is wave-uniform, so these are branches
      Bracket B{0.0, h, S.G0, S.G1};
      if (!P.whole) {
        if (i == P.seg_a) {
          B.tl = P.tau_a;
          B.gl = P.g_a;
        }
        if (i == P.seg_b) {
          B.th = P.tau_b;
          B.gh = P.g_b;
        }
      }
      const double ih = 1.0 / h, sc = (double)s;  // sc: the sign of Im C under (.)^(s)
      for (int k = kA + lane; k <= kB; k += 64) {
        const double f = p.f[k];
        const double w = kTwoPiHi * f;
        const double tau = solve_root(f, dd_, S, B);
        double Er, Ei, gpr, gpi, gcr, gci;
        if constexpr (MIXED) {
          const float2 E = root_E32(f, w, tau, d, ms, ns, S);
          Er = E.x;
          Ei = E.y;
          const float2 gp = ((const float2*)a.g_hp)[k];
          const float2 gc = ((const float2*)a.g_hc)[k];
          gpr = gp.x;
          gpi = gp.y;
          gcr = gc.x;
          gci = gc.y;
        } else {
          const double2 E = root_E64(f, w, tau, d, ms, ns, S);
          Er = E.x;
          Ei = E.y;
          const double2 gp = ((const double2*)a.g_hp)[k];
          const double2 gc = ((const double2*)a.g_hc)[k];
          gpr = gp.x;
          gpi = gp.y;
          gcr = gc.x;
          gci = gc.y;
        }
        // conj(g) E, its imaginary part negated when s > 0 (the sign fold)
        double kpr = gpr * Er + gpi * Ei, kpi = sc * (gpi * Er - gpr * Ei);
        double kxr = gcr * Er + gci * Ei, kxi = sc * (gci * Er - gcr * Ei);
        const double uu = tau * ih;
        double up[7];
        up[0] = 1.0;
        up[1] = uu;
        up[2] = uu * uu;
        up[3] = up[2] * uu;
        up[4] = up[2] * up[2];
        up[5] = up[4] * uu;
        up[6] = up[3] * up[3];
#pragma unroll
        for (int kk = 0; kk < 7; ++kk) {
          acc[2 * kk] += kpr * up[kk];
          acc[2 * kk + 1] += kpi * up[kk];
          acc[14 + 2 * kk] += kxr * up[kk];
          acc[15 + 2 * kk] += kxi * up[kk];
        }
      }
    }
    // the wave's totals; lane r < kVjpMom stores moment r
    double lo16[16], hi16[16];
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      lo16[r] = acc[r];
      hi16[r] = r < kVjpMom - 16 ? acc[16 + r] : 0.0;
    }
    const double tl = wave_sum16(lo16), th = wave_sum16(hi16);
    const int src = (lane < 16 ? lane : lane - 16) * 4;
    const double vl = __shfl(tl, src, 64), vh = __shfl(th, src & 63, 64);
    if (lane < kVjpMom) v.mom[(size_t)c * kVjpMom + lane] = lane < 16 ? vl : vh;
  }
}

// One wave per unit: its chunks' moments summed in chunk order (lane L takes
// chunks L, L + 64, ..., then a fixed-order wave sum), then every row's terms,
// one row per lane.  Every row of the group is written (its other rows have
// no unit of their own).
__global__ __launch_bounds__(256) void vjp_finish_kernel(VjpArgs a, VjpPlan v) {
  const Prepared& p = a.p;
  const int nseg = p.K - 1;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
  const long unit = (long)blockIdx.x * 4 + wave;
  if (unit >= (long)p.Nm * nseg) return;
  const int u = (int)unit;
  const int j = u / nseg, i = u % nseg;
  const bool grouped = p.gsize != nullptr;
  const int g = grouped ? ((const kconst int32_t*)p.gsize)[j] : 1;
  if (g == 0) return;
  const kconst GroupMember* gm = grouped ? (const kconst GroupMember*)p.gmem + j : nullptr;
  const int ch = vjp_chunk_bins(*(const kconst unsigned long long*)v.ctl);
  const int nc = vjp_chunks(((const kconst int32_t*)v.nb)[u], ch);
  const size_t c0 = (size_t)((const kconst int32_t*)v.off)[u];
  double sm[kVjpMom];
#pragma unroll
  for (int r = 0; r < kVjpMom; ++r) sm[r] = 0.0;
  for (int c = lane; c < nc; c += 64) {
    const double* mc = v.mom + (c0 + c) * kVjpMom;
#pragma unroll
    for (int r = 0; r < kVjpMom; ++r) sm[r] += mc[r];
  }
  double lo16[16], hi16[16];
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    lo16[r] = sm[r];
    hi16[r] = r < kVjpMom - 16 ? sm[16 + r] : 0.0;
  }
  const double tl = wave_sum16(lo16), th = wave_sum16(hi16);
  // Q[2k], Q[2k+1] = Qp_k; Q[14 + 2k], Q[15 + 2k] = Qx_k (k = 0..6)
  double Q[kVjpMom];
#pragma unroll
  for (int r = 0; r < kVjpMom; ++r) Q[r] = r < 16 ? __shfl(tl, r * 4, 64) : __shfl(th, (r - 16) * 4, 64);
  const kconst double* kt = (const kconst double*)p.t;
  const double h = kt[i + 1] - kt[i];
  const double hp[4] = {1.0, h, h * h, h * h * h};
  // the group's combined coefficients in u (Cp_j, Cx_j: re, im), in row order,
  // and Z[k] = s sum u^k Im Z over the unit's bins
  double Z[4] = {0.0, 0.0, 0.0, 0.0};
  if (nc > 0) {
    double C[16];
#pragma unroll
    for (int r = 0; r < 16; ++r) C[r] = 0.0;
    const kconst double* kac = (const kconst double*)p.acoef;
    for (int t = 0; t < g; ++t) {
      const int row = grouped ? gm[t].mode : j;
      const ModeConst mt = ((const kconst ModeConst*)p.modes)[row];
      const kconst double* ac = kac + ((size_t)row * nseg + i) * 8;
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const double ar = ac[2 * k] * hp[k], ai = ac[2 * k + 1] * hp[k];
        C[2 * k] += mt.cp_re * ar - mt.cp_im * ai;
        C[2 * k + 1] += mt.cp_re * ai + mt.cp_im * ar;
        C[8 + 2 * k] += mt.cx_re * ar - mt.cx_im * ai;
        C[9 + 2 * k] += mt.cx_re * ai + mt.cx_im * ar;
      }
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) {
#pragma unroll
      for (int jj = 0; jj < 4; ++jj) {
        const int q = jj + k;
        // -Im(conj(C) Q) = C.im Q.re - C.re Q.im
        Z[k] += C[2 * jj + 1] * Q[2 * q] - C[2 * jj] * Q[2 * q + 1];
        Z[k] += C[9 + 2 * jj] * Q[14 + 2 * q] - C[8 + 2 * jj] * Q[15 + 2 * q];
      }
    }
  }
  for (int t = lane; t < g; t += 64) {
    const int row = grouped ? gm[t].mode : j;
    const size_t uo = (size_t)row * nseg + i;
    if (nc == 0) {
      // no bins (or inputs that failed the checks): zero terms, without
      // multiplying coefficients that may not be finite
      if (a.gA) {
#pragma unroll
        for (int q = 0; q < 8; ++q) a.gA[uo * 8 + q] = 0.0;
      }
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        a.Upart[uo * 4 + q] = 0.0;
        a.PZ[uo * 4 + q] = 0.0;
      }
      continue;
    }
    const ModeConst& mt = p.modes[row];
    const double* ac = p.acoef + uo * 8;
    if (a.gA) {
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const double qpr = Q[2 * k], qpi = Q[2 * k + 1], qxr = Q[14 + 2 * k], qxi = Q[15 + 2 * k];
        // conj(c_+) Qp + conj(c_x) Qx
        const double vr = mt.cp_re * qpr + mt.cp_im * qpi + mt.cx_re * qxr + mt.cx_im * qxi;
        const double vi = mt.cp_re * qpi - mt.cp_im * qpr + mt.cx_re * qxi - mt.cx_im * qxr;
        a.gA[uo * 8 + 2 * k] = hp[k] * vr;
        a.gA[uo * 8 + 2 * k + 1] = hp[k] * vi;
      }
    }
    // sum_j a^_j conj(Q_j)
    double upr = 0.0, upi = 0.0, uxr = 0.0, uxi = 0.0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const double ar = ac[2 * k] * hp[k], ai = ac[2 * k + 1] * hp[k];
      upr += ar * Q[2 * k] + ai * Q[2 * k + 1];
      upi += ai * Q[2 * k] - ar * Q[2 * k + 1];
      uxr += ar * Q[14 + 2 * k] + ai * Q[15 + 2 * k];
      uxi += ai * Q[14 + 2 * k] - ar * Q[15 + 2 * k];
    }
    a.Upart[uo * 4 + 0] = upr;
    a.Upart[uo * 4 + 1] = upi;
    a.Upart[uo * 4 + 2] = uxr;
    a.Upart[uo * 4 + 3] = uxi;
#pragma unroll
    for (int k = 0; k < 4; ++k) a.PZ[uo * 4 + k] = t == 0 ? hp[k] * Z[k] : 0.0;
  }
}

// gPhi[0][i][k] = sum_mu m_mu PZ[mu][i][k], gPhi[1][i][k] = sum_mu n_mu PZ[mu][i][k]
__global__ __launch_bounds__(256) void vjp_phi_kernel(int Nm, int nseg, const ModeConst* __restrict__ modes,
                                                      const double* __restrict__ PZ, double* __restrict__ gPhi) {
  __shared__ double red[8][256];
  const int i = blockIdx.x;
  double v[8];
#pragma unroll
  for (int q = 0; q < 8; ++q) v[q] = 0.0;
  for (int mu = threadIdx.x; mu < Nm; mu += blockDim.x) {
    const double m = modes[mu].m, n = modes[mu].n;
    const double* z = PZ + ((size_t)mu * nseg + i) * 4;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      v[k] += m * z[k];
      v[4 + k] += n * z[k];
    }
  }
#pragma unroll
  for (int q = 0; q < 8; ++q) red[q][threadIdx.x] = v[q];
  __syncthreads();
  for (int w = blockDim.x / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w)
#pragma unroll
      for (int q = 0; q < 8; ++q) red[q][threadIdx.x] += red[q][threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x < 8) {
    const int q = threadIdx.x;
    gPhi[((size_t)(q / 4) * nseg + i) * 4 + (q % 4)] = red[q][0];
  }
}

// Per mode: U = sum over segments; contributions to dL/dtheta, dL/dphi, dL/dscale.
__global__ __launch_bounds__(64) void vjp_modes_kernel(int Nm, int nseg, const int32_t* __restrict__ l,
                                                       const int32_t* __restrict__ mm, double theta, double phi,
                                                       double scale, uint32_t flags, const ModeConst* __restrict__ modes,
                                                       const double* __restrict__ Upart, double* __restrict__ T3) {
  const int mu = blockIdx.x * blockDim.x + threadIdx.x;
  if (mu >= Nm) return;
  double u[4] = {0.0, 0.0, 0.0, 0.0};
  for (int i = 0; i < nseg; ++i) {
    const double* up = Upart + ((size_t)mu * nseg + i) * 4;
#pragma unroll
    for (int q = 0; q < 4; ++q) u[q] += up[q];
  }
  const int li = l[mu], mi = mm[mu];
  const double4 y = swsh_m2_with_dtheta(li, mi, theta, phi);
  double4 yp = make_double4(0.0, 0.0, 0.0, 0.0);  // (-1)^l conj(Y_{l,-m}) and its theta derivative
  if (mi > 0 && !(flags & FDEMRI_NO_PARTNERS)) {
    const double4 ym = swsh_m2_with_dtheta(li, -mi, theta, phi);
    const double sg = (li & 1) ? -1.0 : 1.0;
    yp = make_double4(sg * ym.x, -sg * ym.y, sg * ym.z, -sg * ym.w);
  }
  // unit-scale factors cu_+ = (Y + Yp)/2, cu_x = i (Y - Yp)/2 and their theta derivatives
  const double cpr = 0.5 * (y.x + yp.x), cpi = 0.5 * (y.y + yp.y);
  const double cxr = -0.5 * (y.y - yp.y), cxi = 0.5 * (y.x - yp.x);
  const double dpr = 0.5 * (y.z + yp.z), dpi = 0.5 * (y.w + yp.w);
  const double dxr = -0.5 * (y.w - yp.w), dxi = 0.5 * (y.z - yp.z);
  auto re_mul = [](double ar, double ai, double br, double bi) { return ar * br - ai * bi; };
  const double g_scale = re_mul(u[0], u[1], cpr, cpi) + re_mul(u[2], u[3], cxr, cxi);
  const double g_theta = scale * (re_mul(u[0], u[1], dpr, dpi) + re_mul(u[2], u[3], dxr, dxi));
  // d c / d phi = i m c
  const double mphi = (double)mi * scale;
  const double g_phi = mphi * (re_mul(u[0], u[1], -cpi, cpr) + re_mul(u[2], u[3], -cxi, cxr));
  double* o = T3 + (size_t)mu * 4;
  o[0] = g_theta;
  o[1] = g_phi;
  o[2] = g_scale;
  o[3] = 0.0;
}

// g_scalars = [sum_mu T3 (theta, phi, scale), sum_i gPhi[0][i][0], sum_i gPhi[1][i][0]]
__global__ __launch_bounds__(256) void vjp_final_kernel(int Nm, int nseg, const double* __restrict__ T3,
                                                        const double* __restrict__ gPhi, double* __restrict__ out) {
  __shared__ double red[5][256];
  double v[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
  for (int mu = threadIdx.x; mu < Nm; mu += blockDim.x) {
    v[0] += T3[(size_t)mu * 4 + 0];
    v[1] += T3[(size_t)mu * 4 + 1];
    v[2] += T3[(size_t)mu * 4 + 2];
  }
  for (int i = threadIdx.x; i < nseg; i += blockDim.x) {
    v[3] += gPhi[((size_t)0 * nseg + i) * 4];
    v[4] += gPhi[((size_t)1 * nseg + i) * 4];
  }
#pragma unroll
  for (int q = 0; q < 5; ++q) red[q][threadIdx.x] = v[q];
  __syncthreads();
  for (int w = blockDim.x / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w)
#pragma unroll
      for (int q = 0; q < 5; ++q) red[q][threadIdx.x] += red[q][threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x < 5) out[threadIdx.x] = red[threadIdx.x][0];
}

// Transposed not-a-knot spline: gradient w.r.t. knot values from the
// gradient w.r.t. segment coefficients (the adjoint of the slope solve of the
// spline kernel: coefficient terms -> slope and divided-difference adjoints,
// a transposed tridiagonal solve by parallel cyclic reduction, then the
// divided differences back to knots).  One workgroup per real series:
// series 0, 1 = Phi_phi, Phi_r; 2 + 2 mu + part = amplitude mode mu (re, im).
template <int NT>
__global__ __launch_bounds__(NT) void spline_adjoint_kernel(int K, const double* __restrict__ t, int Nm,
                                                            const double* __restrict__ gPhi_coef,
                                                            const double* __restrict__ gA_coef,
                                                            double* __restrict__ gPhi_knots,
                                                            double* __restrict__ gA_knots,
                                                            const int32_t* __restrict__ status) {
  __shared__ double sa[NT], sb[NT], sc[NT], sr[NT], sh[NT], sdb[NT];
  const int i = threadIdx.x;
  const int series = blockIdx.x;
  const int n = K - 1;
  const bool amp = series >= 2;
  if (!amp && gPhi_knots == nullptr) return;
  if (amp && gA_knots == nullptr) return;
  const int mode = amp ? (series - 2) >> 1 : 0, part = amp ? (series - 2) & 1 : 0;
  if (*status != 0) {
    // inputs that failed the checks (the knots may not even be increasing):
    // a zero gradient, without the solve
    if (i < K) {
      if (amp)
        gA_knots[((size_t)mode * K + i) * 2 + part] = 0.0;
      else
        gPhi_knots[(size_t)series * K + i] = 0.0;
    }
    return;
  }
  auto gcoef = [&](int seg, int k) -> double {
    if (amp) return gA_coef[(((size_t)mode * n + seg) * 4 + k) * 2 + part];
    return gPhi_coef[((size_t)series * n + seg) * 4 + k];
  };
  if (i < n) sh[i] = t[i + 1] - t[i];
  __syncthreads();
  // transposed tridiagonal rows: sub = c_{i-1}, diag = b_i, super = a_{i+1} of the forward matrix
  auto fa = [&](int j) -> double {  // forward sub-diagonal a_j
    if (j <= 0 || j > n) return 0.0;
    if (j == n) return sh[n - 2] + sh[n - 1];
    return sh[j];
  };
  auto fb = [&](int j) -> double {
    if (j == 0) return sh[1];
    if (j == n) return sh[n - 2];
    return 2.0 * (sh[j - 1] + sh[j]);
  };
  auto fc = [&](int j) -> double {  // forward super-diagonal c_j
    if (j < 0 || j >= n) return 0.0;
    if (j == 0) return sh[0] + sh[1];
    return sh[j - 1];
  };
  double a = 0.0, b = 1.0, c = 0.0, r = 0.0;
  double dbar = 0.0;
  if (i < K) {
    a = (i >= 1) ? fc(i - 1) : 0.0;
    b = fb(i);
    c = (i <= n - 1) ? fa(i + 1) : 0.0;
    double v = 0.0;
    if (i < n) {
      const double h = sh[i];
      v += gcoef(i, 1) - 2.0 * gcoef(i, 2) / h + gcoef(i, 3) / (h * h);
      dbar = 3.0 * gcoef(i, 2) / h - 2.0 * gcoef(i, 3) / (h * h);
    }
    if (i >= 1) {
      const double h = sh[i - 1];
      v += -gcoef(i - 1, 2) / h + gcoef(i - 1, 3) / (h * h);
    }
    r = v;
  }
  sa[i] = a;
  sb[i] = b;
  sc[i] = c;
  sr[i] = r;
  __syncthreads();
  for (int s = 1; s < NT; s <<= 1) {
    const int im = i - s, ip = i + s;
    double am = 0.0, bm = 1.0, cm = 0.0, rm = 0.0, ap = 0.0, bp = 1.0, cp = 0.0, rp = 0.0;
    if (im >= 0) {
      am = sa[im];
      bm = sb[im];
      cm = sc[im];
      rm = sr[im];
    }
    if (ip < NT) {
      ap = sa[ip];
      bp = sb[ip];
      cp = sc[ip];
      rp = sr[ip];
    }
    const double k1 = a / bm, k2 = c / bp;
    const double na = -am * k1, nc = -cp * k2, nb = b - cm * k1 - ap * k2, nr = r - rm * k1 - rp * k2;
    __syncthreads();
    a = na;
    b = nb;
    c = nc;
    r = nr;
    sa[i] = a;
    sb[i] = b;
    sc[i] = c;
    sr[i] = r;
    __syncthreads();
  }
  const double rbar = r / b;
  __syncthreads();
  sr[i] = rbar;
  __syncthreads();
  // divided-difference adjoints
  if (i < n) {
    double v = 0.0;
    if (i == 0) v += (2.0 * sh[1] * sh[1] + 3.0 * sh[0] * sh[1]) / (sh[0] + sh[1]) * sr[0];
    if (i >= 1 && i <= n - 1) v += 3.0 * sh[i - 1] * sr[i];
    if (i + 1 <= n - 1) v += 3.0 * sh[i + 1] * sr[i + 1];
    if (i == 1) v += sh[0] * sh[0] / (sh[0] + sh[1]) * sr[0];
    if (i == n - 2) v += sh[n - 1] * sh[n - 1] / (sh[n - 2] + sh[n - 1]) * sr[n];
    if (i == n - 1) v += (2.0 * sh[n - 2] * sh[n - 2] + 3.0 * sh[n - 2] * sh[n - 1]) / (sh[n - 2] + sh[n - 1]) * sr[n];
    dbar += v;
  }
  sdb[i] = dbar;
  __syncthreads();
  if (i < K) {
    double y = (i < n) ? gcoef(i, 0) : 0.0;
    if (i >= 1) y += sdb[i - 1] / sh[i - 1];
    if (i < n) y -= sdb[i] / sh[i];
    if (amp)
      gA_knots[((size_t)mode * K + i) * 2 + part] = y;
    else
      gPhi_knots[(size_t)series * K + i] = y;
  }
}

// The most chunks a call can have (units plus kVjpChunkCap: the chunk size
// grows with the total bins to keep within it) and the bytes of their moments.
long vjp_max_chunks(long units) { return units + kVjpChunkCap; }
size_t vjp_mom_bytes(long units) { return (size_t)vjp_max_chunks(units) * kVjpMom * sizeof(double); }

// Bytes of device scratch the chunk-offset scan needs for `units` units.
size_t vjp_scan_bytes(long units) {
  size_t bytes = 0;
  auto in = rocprim::make_transform_iterator(rocprim::make_counting_iterator(0), VjpChunkCount{nullptr, nullptr});
  (void)rocprim::exclusive_scan(nullptr, bytes, in, (int32_t*)nullptr, 0, (size_t)units, rocprim::plus<int>());
  return bytes;
}

// The adjoint's bin work: plan, chunk offsets, chunks, and the per-unit sums
// into gA_coef, PZ and Upart.
hipError_t launch_vjp_units(const Prepared& p, const float* acoef32, bool mixed, const void* g_hp, const void* g_hc,
                            double* gA_coef, double* PZ, double* Upart, int2* rng, int32_t* nb, int32_t* off,
                            unsigned long long* ctl, int32_t* unit_of, double* mom, void* scan_tmp,
                            size_t scan_bytes, hipStream_t stream) {
  VjpArgs a;
  a.p = p;
  a.acoef32 = acoef32;
  a.g_hp = g_hp;
  a.g_hc = g_hc;
  a.gA = gA_coef;
  a.PZ = PZ;
  a.Upart = Upart;
  VjpPlan v{rng, nb, off, ctl, unit_of, mom};
  const int nseg = p.K - 1;
  const long units = (long)p.Nm * nseg;
  vjp_plan_zero_kernel<<<1, 1, 0, stream>>>(ctl);
  vjp_plan_kernel<<<(unsigned)((units + 255) / 256), 256, 0, stream>>>(p, v);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  auto in = rocprim::make_transform_iterator(rocprim::make_counting_iterator(0), VjpChunkCount{nb, ctl});
  size_t bytes = scan_bytes;
  e = rocprim::exclusive_scan(scan_tmp, bytes, in, off, 0, (size_t)units, rocprim::plus<int>(), stream);
  if (e != hipSuccess) return e;
  vjp_map_kernel<<<(unsigned)((units + 255) / 256), 256, 0, stream>>>((int)units, v);
  // as many waves as the device holds at the kernel's occupancy; the chunks
  // are handed out, so more would only find the counter exhausted
  int dev = 0, ncu = 0;
  e = hipGetDevice(&dev);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
  if (e != hipSuccess) return e;
  if (mixed)
    vjp_chunk_kernel<true><<<(unsigned)(ncu * vjp_min_waves<true>()), 256, 0, stream>>>(a, v);
  else
    vjp_chunk_kernel<false><<<(unsigned)(ncu * vjp_min_waves<false>()), 256, 0, stream>>>(a, v);
  vjp_finish_kernel<<<(unsigned)((units + 3) / 4), 256, 0, stream>>>(a, v);
  return hipGetLastError();
}

// The reductions after the chunk sums: phase-coefficient gradients, per-mode
// angle and scale terms, and the five scalars.
hipError_t launch_vjp_reduce(const Prepared& p, double* PZ, double* Upart, double* T3, double* gPhi_coef,
                             double* g_scalars, const int32_t* l, const int32_t* m, double theta, double phi,
                             double scale, uint32_t flags, hipStream_t stream) {
  const int nseg = p.K - 1;
  vjp_phi_kernel<<<nseg, 256, 0, stream>>>(p.Nm, nseg, p.modes, PZ, gPhi_coef);
  vjp_modes_kernel<<<(p.Nm + 63) / 64, 64, 0, stream>>>(p.Nm, nseg, l, m, theta, phi, scale, flags, p.modes, Upart, T3);
  vjp_final_kernel<<<1, 256, 0, stream>>>(p.Nm, nseg, T3, gPhi_coef, g_scalars);
  return hipGetLastError();
}

hipError_t launch_spline_adjoint(int K, const double* t, int Nm, const double* gPhi_coef, const double* gA_coef,
                                 double* gPhi_knots, double* gA_knots, const int32_t* status, hipStream_t stream) {
  dim3 grid(2 + 2 * Nm);
  if (K <= 64)
    spline_adjoint_kernel<64><<<grid, 64, 0, stream>>>(K, t, Nm, gPhi_coef, gA_coef, gPhi_knots, gA_knots, status);
  else if (K <= 128)
    spline_adjoint_kernel<128><<<grid, 128, 0, stream>>>(K, t, Nm, gPhi_coef, gA_coef, gPhi_knots, gA_knots, status);
  else if (K <= 256)
    spline_adjoint_kernel<256><<<grid, 256, 0, stream>>>(K, t, Nm, gPhi_coef, gA_coef, gPhi_knots, gA_knots, status);
  else
    spline_adjoint_kernel<512><<<grid, 512, 0, stream>>>(K, t, Nm, gPhi_coef, gA_coef, gPhi_knots, gA_knots, status);
  return hipGetLastError();
}

}  // namespace fdemri
