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
// The forward terms are recomputed, not stored: one wavefront per
// (voice group, spline segment) re-evaluates the roots of every bin whose
// root lies in that segment (the same segment assignment, bracket and
// arithmetic as the forward gather), reduces moments of conj(g) E in
// registers, and forms every row's terms from them.  All further reductions
// run in a fixed order, so the gradient is deterministic and no atomics are
// used.
#include "evalcore.hpp"
#include "harmonics.hpp"
#include "search.hpp"

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

// Occupancy target in waves per SIMD: the mixed adjoint fits 4 (a few spills
// outside the bin loop); the FP64 one would spill inside it and stays at 3.
template <bool MIXED>
constexpr int vjp_min_waves() {
  return MIXED ? 4 : 3;
}

// One unit per (voice group, spline segment): the group at sorted position j
// (its first row; every row its own group when the table is not grouped) and
// segment i.  The rows of a group share the pieces, roots and E, so the bin
// loop forms, per piece, the moments
//   Mp_k = sum over bins of u^k conj(g_+) E,  Mx_k = sum u^k conj(g_x) E,
//   Y_k  = sum u^k Im Z,  Z = conj(g_+) Cp(u)^(s) E + conj(g_x) Cx(u)^(s) E,
// u = tau / h, k = 0..3, with Cp(u) = sum_t c_+,t A_t (Cx likewise) the
// group's combined amplitude, and every row's terms follow after the loop (a
// the row's amplitude coefficients in u, a^_j = a_j h^j, c its factors):
//   s > 0: dL/da_k = h^k conj(c_+ Mp_k + c_x Mx_k),  U_+ = sum_j a^_j Mp_j,
//   s < 0: dL/da_k = h^k (conj(c_+) Mp_k + conj(c_x) Mx_k),  U_+ = sum_j a^_j conj(Mp_j)
// (U_x likewise with Mx), and the group's sum s tau^k Im Z = s h^k Y_k
// ((.)^(s): conjugate when s < 0).  The bins a unit evaluates are those of
// the per-row form (the same segment assignment, bracket and root).  Outputs
// per row of the group: gA (8), Upart (4) and PZ (4; the group's sum at its
// first row, zero at the others, since the phase gradient sums m PZ over
// the rows).
template <bool MIXED>
__global__ __launch_bounds__(256, vjp_min_waves<MIXED>()) void vjp_unit_kernel(VjpArgs a) {
  // each wave's combined coefficients Cp, Cx in u (re, im per power)
  __shared__ double comb[4][16];
  const Prepared& p = a.p;
  const int nseg = p.K - 1;
  // the wave index is uniform; in a scalar register it makes the unit, and
  // every load indexed by it, scalar
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
  const long unit = (long)blockIdx.x * 4 + wave;
  if (unit >= (long)p.Nm * nseg) return;
  const int j = (int)(unit / nseg), i = (int)(unit % nseg);
  const bool grouped = p.gsize != nullptr;
  const int g = grouped ? ((const kconst int32_t*)p.gsize)[j] : 1;
  if (g == 0) return;  // a group's other rows: their outputs are this group's unit's
  const kconst GroupMember* gm = grouped ? (const kconst GroupMember*)p.gmem + j : nullptr;
  const int lead = grouped ? gm[0].mode : j;
  const ModeConst md = ((const kconst ModeConst*)p.modes)[lead];
  const double m = md.m, n = md.n;

  // segment data of this unit (wave-uniform; read-only tables through the
  // constant address space, so scalar loads)
  const kconst double* kt = (const kconst double*)p.t;
  const kconst double* kFp = (const kconst double*)p.Fphi;
  const kconst double* kFr = (const kconst double*)p.Fr;
  const double ti = kt[i], h = kt[i + 1] - ti;
  const double F0 = knot_freq(m, kFp[i], n, kFr[i]);
  const double F1 = knot_freq(m, kFp[i + 1], n, kFr[i + 1]);
  const kconst double* cFp = (const kconst double*)p.tcoef + ((size_t)0 * nseg + i) * 4;
  const kconst double* cFr = (const kconst double*)p.tcoef + ((size_t)1 * nseg + i) * 4;
  const kconst double* cPp = (const kconst double*)p.tcoef + ((size_t)2 * nseg + i) * 4;
  const kconst double* cPr = (const kconst double*)p.tcoef + ((size_t)3 * nseg + i) * 4;
  const double Ppr = reduce_2pi(((const kconst double*)p.Phiphi)[i]);
  const double Prr = reduce_2pi(((const kconst double*)p.Phir)[i]);
  const double hp[4] = {1.0, h, h * h, h * h * h};
  auto row_of = [&](int t) { return grouped ? gm[t].mode : j; };

  // every row's outputs start at zero (each row's by the lane that adds to
  // them); lanes 0..15 form the group's combined coefficients, in row order
  double cv = 0.0;
  for (int t = 0; t < g; ++t) {
    const int row = row_of(t);
    if (lane < 16) {
      const ModeConst& mt = p.modes[row];
      const int k = (lane & 7) >> 1;
      const double* ac = p.acoef + ((size_t)row * nseg + i) * 8 + 2 * k;
      const double ar = ac[0] * hp[k], ai = ac[1] * hp[k];
      const double cr = lane < 8 ? mt.cp_re : mt.cx_re, ci = lane < 8 ? mt.cp_im : mt.cx_im;
      cv += (lane & 1) ? cr * ai + ci * ar : cr * ar - ci * ai;
    }
  }
  if (lane < 16) comb[wave][lane] = cv;  // read by the same wave after the fence below
  for (int t = lane; t < g; t += 64) {
    const size_t u = (size_t)row_of(t) * nseg + i;
    if (a.gA) {
#pragma unroll
      for (int q = 0; q < 8; ++q) a.gA[u * 8 + q] = 0.0;
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      a.Upart[u * 4 + q] = 0.0;
      a.PZ[u * 4 + q] = 0.0;
    }
  }
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
  const double* cb = comb[wave];
  double pz[4] = {0.0, 0.0, 0.0, 0.0};

  // a waveform whose inputs failed the checks has a zero gradient
  const int npieces = *(const kconst int32_t*)p.status != 0 ? 0 : md.npieces;
  for (int q = 0; q < npieces; ++q) {
    const Piece P = ((const kconst Piece*)p.pieces)[(size_t)lead * kMaxPieces + q];
    if (i < P.seg_a || i > P.seg_b || P.k_lo > P.k_hi) continue;
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
    // bins whose root the forward search places in segment i of this piece:
    // the largest segment j in [seg_a, seg_b] with j == seg_a or d g_j < d f
    int kA = P.k_lo, kB = P.k_hi;
    const double gi = S.G0, gi1 = S.G1;
    if (d > 0) {
      if (i > P.seg_a) kA = max(kA, first_gt(p.f, p.Nf, gi));
      if (i < P.seg_b) kB = min(kB, first_gt(p.f, p.Nf, gi1) - 1);
    } else {
      if (i > P.seg_a) kB = min(kB, first_ge(p.f, p.Nf, gi) - 1);
      if (i < P.seg_b) kA = max(kA, first_ge(p.f, p.Nf, gi1));
    }
    if (kA > kB) continue;
    const Bracket B = make_bracket(P, i, S);
    const double ih = 1.0 / h, sc = (double)s;  // sc: the sign of Im C under (.)^(s)
    // moments: acc[2k], acc[2k+1] = Mp_k; acc[8 + 2k], acc[9 + 2k] = Mx_k; acc[16 + k] = Y_k
    double acc[20];
#pragma unroll
    for (int r = 0; r < 20; ++r) acc[r] = 0.0;
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
      // conj(g) E
      double kpr = gpr * Er + gpi * Ei, kpi = gpr * Ei - gpi * Er;
      double kxr = gcr * Er + gci * Ei, kxi = gcr * Ei - gci * Er;
      const double u = tau * ih;
      // the combined amplitudes at u, conjugated when s < 0
      const double apr = cb[0] + u * (cb[2] + u * (cb[4] + u * cb[6]));
      const double api = sc * (cb[1] + u * (cb[3] + u * (cb[5] + u * cb[7])));
      const double axr = cb[8] + u * (cb[10] + u * (cb[12] + u * cb[14]));
      const double axi = sc * (cb[9] + u * (cb[11] + u * (cb[13] + u * cb[15])));
      double imz = (kpr * api + kpi * apr) + (kxr * axi + kxi * axr);
#pragma unroll
      for (int kk = 0; kk < 4; ++kk) {
        acc[2 * kk] += kpr;
        acc[2 * kk + 1] += kpi;
        acc[8 + 2 * kk] += kxr;
        acc[9 + 2 * kk] += kxi;
        acc[16 + kk] += imz;
        kpr *= u;
        kpi *= u;
        kxr *= u;
        kxi *= u;
        imz *= u;
      }
    }
    // the wave's totals, in every lane
    double lo16[16], hi16[16];
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      lo16[r] = acc[r];
      hi16[r] = r < 4 ? acc[16 + r] : 0.0;
    }
    const double tl = wave_sum16(lo16), th = wave_sum16(hi16);
    double M[16];
#pragma unroll
    for (int r = 0; r < 16; ++r) M[r] = __shfl(tl, r * 4, 64);
#pragma unroll
    for (int k = 0; k < 4; ++k) pz[k] += sc * hp[k] * __shfl(th, k * 4, 64);
    const bool pos = s > 0;
    // every row's terms, one row per lane
    for (int t = lane; t < g; t += 64) {
      const int row = row_of(t);
      const size_t uo = (size_t)row * nseg + i;
      const ModeConst& mt = p.modes[row];
      const double* ac = p.acoef + uo * 8;
      if (a.gA) {
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          const double mpr = M[2 * k], mpi = M[2 * k + 1], mxr = M[8 + 2 * k], mxi = M[9 + 2 * k];
          double vr, vi;
          if (pos) {
            // conj(c_+ Mp + c_x Mx)
            vr = mt.cp_re * mpr - mt.cp_im * mpi + mt.cx_re * mxr - mt.cx_im * mxi;
            vi = -(mt.cp_re * mpi + mt.cp_im * mpr + mt.cx_re * mxi + mt.cx_im * mxr);
          } else {
            // conj(c_+) Mp + conj(c_x) Mx
            vr = mt.cp_re * mpr + mt.cp_im * mpi + mt.cx_re * mxr + mt.cx_im * mxi;
            vi = mt.cp_re * mpi - mt.cp_im * mpr + mt.cx_re * mxi - mt.cx_im * mxr;
          }
          a.gA[uo * 8 + 2 * k] += hp[k] * vr;
          a.gA[uo * 8 + 2 * k + 1] += hp[k] * vi;
        }
      }
      double upr = 0.0, upi = 0.0, uxr = 0.0, uxi = 0.0;
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const double ar = ac[2 * k] * hp[k], ai = ac[2 * k + 1] * hp[k];
        const double mpr = M[2 * k], mpi = pos ? M[2 * k + 1] : -M[2 * k + 1];
        const double mxr = M[8 + 2 * k], mxi = pos ? M[9 + 2 * k] : -M[9 + 2 * k];
        upr += ar * mpr - ai * mpi;
        upi += ar * mpi + ai * mpr;
        uxr += ar * mxr - ai * mxi;
        uxi += ar * mxi + ai * mxr;
      }
      a.Upart[uo * 4 + 0] += upr;
      a.Upart[uo * 4 + 1] += upi;
      a.Upart[uo * 4 + 2] += uxr;
      a.Upart[uo * 4 + 3] += uxi;
    }
  }
  if (lane == 0) {
    const size_t u = (size_t)lead * nseg + i;
#pragma unroll
    for (int k = 0; k < 4; ++k) a.PZ[u * 4 + k] = pz[k];
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

// The per-(mode, segment) unit kernel of the adjoint (its partial sums into
// gA_coef, PZ and Upart).
hipError_t launch_vjp_units(const Prepared& p, const float* acoef32, bool mixed, const void* g_hp, const void* g_hc,
                            double* gA_coef, double* PZ, double* Upart, hipStream_t stream) {
  VjpArgs a;
  a.p = p;
  a.acoef32 = acoef32;
  a.g_hp = g_hp;
  a.g_hc = g_hc;
  a.gA = gA_coef;
  a.PZ = PZ;
  a.Upart = Upart;
  const int nseg = p.K - 1;
  const long units = (long)p.Nm * nseg;
  const unsigned blocks = (unsigned)((units + 3) / 4);
  if (mixed)
    vjp_unit_kernel<true><<<blocks, 256, 0, stream>>>(a);
  else
    vjp_unit_kernel<false><<<blocks, 256, 0, stream>>>(a);
  return hipGetLastError();
}

// The reductions after the unit kernel: phase-coefficient gradients, per-mode
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
