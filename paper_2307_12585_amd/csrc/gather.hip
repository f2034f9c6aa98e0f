// Frequency-domain mode sum (Sec. 2.2, Eqs. cubic_equation, SPAintegral2,
// extendedspa1), bin-major.
//
// The paper's GPU kernel places one block per (voice, spline segment) and
// adds every contribution atomically into the output vector.  Here each
// wavefront owns a tile of contiguous frequency bins instead and gathers all
// contributions to its bins in registers, so every output element is written
// once, coalesced, in a fixed order of voices and pieces (deterministic, no
// atomics):
//   1. the workgroup stages the shared trajectory tables (knots and spline
//      coefficients of F_phi, F_r, Phi_phi, Phi_r) in LDS;
//   2. the wave scans the per-mode bin ranges 64 modes at a time and keeps,
//      by ballot, the modes whose range meets its tile;
//   3. for each active piece of an active mode, each lane with a bin inside
//      the piece's range finds the spline segment holding f (binary search
//      over the knot frequencies), solves the cubic of Eq. cubic_equation for
//      the root by safeguarded Newton iteration, evaluates dF/dt, d2F/dt2,
//      the factor G of Eq. extendedspa1, the phase 2 pi f t - Phi_V(t) (large
//      part in double-double, reduced modulo 2 pi) and the amplitude spline,
//      and accumulates h_+ and h_x;
//   4. the wave stores its tile.
// FP64 path: everything in double.  Mixed path: root, derivatives, phase and
// its reduction in double; the special function, sincos, amplitude spline and
// products in float with compensated (Kahan) accumulation.
#include "evalcore.hpp"

namespace fdemri {

struct GatherArgs {
  Prepared p;
  const float* acoef32;  // [Nm][K-1][8] normalised-u amplitude coefficients (mixed path)
  void* hp;
  void* hc;
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
  float v[4], c[4];
  __device__ __forceinline__ void zero() {
#pragma unroll
    for (int q = 0; q < 4; ++q) v[q] = c[q] = 0.f;
  }
  __device__ __forceinline__ void add(int q, float y) {
    // compensated (Kahan) summation
    const float yy = y - c[q];
    const float tt = v[q] + yy;
    c[q] = (tt - v[q]) - yy;
    v[q] = tt;
  }
};

struct Lds {
  const double* t;
  const double* Fp;
  const double* Fr;
  const double* Pp;
  const double* Pr;
  const double* cF;  // [K-1][6]: Fphi c1..c3, Fr c1..c3
  const double* cP;  // [K-1][6]: Phiphi c1..c3, Phir c1..c3
};

// One (bin, piece) evaluation.  The spline segment holding f is the largest i
// in [seg_a, seg_b] whose start value precedes f in the direction of the
// piece (i == seg_a or d g_i < d f; ties go to the lower segment); it is found
// from the piece's rate guess and a short correction in either direction.
template <bool MIXED>
__device__ __forceinline__ void eval_bin(const double f, const Piece& P, const double m, const double n,
                                         const double cpr, const double cpi, const double cxr, const double cxi,
                                         const double* __restrict__ ac, const float* __restrict__ ac32,
                                         const Lds& L, Acc<MIXED>& acc) {
  const int s = P.s, d = P.d;
  const double sd = (double)s;
  const double dd_ = (double)d;
  const double span = (double)(P.seg_b - P.seg_a);
  const double est = fmin(fmax((f - P.g_a) * (double)P.rate, 0.0), span);
  int i = P.seg_a + (int)est;
  while (i > P.seg_a && !(dd_ * (sd * knot_freq(m, L.Fp[i], n, L.Fr[i])) < dd_ * f)) --i;
  while (i < P.seg_b && dd_ * (sd * knot_freq(m, L.Fp[i + 1], n, L.Fr[i + 1])) < dd_ * f) ++i;
  SegData S;
  S.ti = L.t[i];
  S.h = L.t[i + 1] - S.ti;
  S.F0 = knot_freq(m, L.Fp[i], n, L.Fr[i]);
  S.F1 = knot_freq(m, L.Fp[i + 1], n, L.Fr[i + 1]);
  const double* cf = L.cF + i * 6;
  S.a1 = m * cf[0] + n * cf[3];
  S.a2 = m * cf[1] + n * cf[4];
  S.a3 = m * cf[2] + n * cf[5];
  const double* cp = L.cP + i * 6;
  S.b1 = m * cp[0] + n * cp[3];
  S.b2 = m * cp[1] + n * cp[4];
  S.b3 = m * cp[2] + n * cp[5];
  S.Ppi = L.Pp[i];
  S.Pri = L.Pr[i];
  const Bracket B = make_bracket(P, i, sd, S);
  const double tau = solve_root(f, sd, dd_, S, B);

  if constexpr (!MIXED) {
    double2 E, A;
    root_terms64(f, tau, sd, d, m, n, S, ac + (size_t)i * 8, E, A);
    double pr = A.x * cpr - A.y * cpi, pi = A.x * cpi + A.y * cpr;
    double xr = A.x * cxr - A.y * cxi, xi = A.x * cxi + A.y * cxr;
    if (s < 0) {
      pi = -pi;
      xi = -xi;
    }
    acc.v[0] += pr * E.x - pi * E.y;
    acc.v[1] += pr * E.y + pi * E.x;
    acc.v[2] += xr * E.x - xi * E.y;
    acc.v[3] += xr * E.y + xi * E.x;
  } else {
    float2 E, A;
    root_terms32(f, tau, sd, d, m, n, S, ac32 + (size_t)i * 8, E, A);
    const float fcpr = (float)cpr, fcpi = (float)cpi, fcxr = (float)cxr, fcxi = (float)cxi;
    float pr = A.x * fcpr - A.y * fcpi, pi = A.x * fcpi + A.y * fcpr;
    float xr = A.x * fcxr - A.y * fcxi, xi = A.x * fcxi + A.y * fcxr;
    if (s < 0) {
      pi = -pi;
      xi = -xi;
    }
    acc.add(0, pr * E.x - pi * E.y);
    acc.add(1, pr * E.y + pi * E.x);
    acc.add(2, xr * E.x - xi * E.y);
    acc.add(3, xr * E.y + xi * E.x);
  }
}

// Cooperative copy of one waveform's shared trajectory tables into LDS
// (caller synchronises).
__device__ __forceinline__ Lds stage_lds(const Prepared& p, double* lds) {
  const int K = p.K, nseg = K - 1;
  double* s_t = lds;
  double* s_Fp = s_t + K;
  double* s_Fr = s_Fp + K;
  double* s_Pp = s_Fr + K;
  double* s_Pr = s_Pp + K;
  double* s_cF = s_Pr + K;
  double* s_cP = s_cF + 6 * nseg;
  for (int i = threadIdx.x; i < K; i += blockDim.x) {
    s_t[i] = p.t[i];
    s_Fp[i] = p.Fphi[i];
    s_Fr[i] = p.Fr[i];
    s_Pp[i] = p.Phiphi[i];
    s_Pr[i] = p.Phir[i];
  }
  for (int i = threadIdx.x; i < nseg; i += blockDim.x) {
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      s_cF[i * 6 + c] = p.tcoef[((size_t)0 * nseg + i) * 4 + 1 + c];
      s_cF[i * 6 + 3 + c] = p.tcoef[((size_t)1 * nseg + i) * 4 + 1 + c];
      s_cP[i * 6 + c] = p.tcoef[((size_t)2 * nseg + i) * 4 + 1 + c];
      s_cP[i * 6 + 3 + c] = p.tcoef[((size_t)3 * nseg + i) * 4 + 1 + c];
    }
  }
  return Lds{s_t, s_Fp, s_Fr, s_Pp, s_Pr, s_cF, s_cP};
}

// Zeros for the tile [k0, k0 + 64 BPL) (blocks outside every voice's range).
template <bool MIXED, int BPL, int WAVES>
__device__ __forceinline__ void zero_tile(void* hp, void* hc, int Nf, long k0) {
  for (int t = threadIdx.x; t < 64 * BPL; t += 64 * WAVES) {
    const long k = k0 + t;
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

// One workgroup's tile of 64 * BPL contiguous bins starting at k0.  Every
// wave enumerates the (mode, piece) pairs active in the tile and evaluates
// those with (mode + piece) % WAVES == its index; each lane accumulates its
// bins in registers, and the partial sums are added in LDS in a fixed wave
// order.  The grouping and the order within a group depend only on the
// (mode, piece) pair, so the result is independent of scheduling and of the
// tile size.  red: LDS scratch of WAVES * BPL * 64 * 4 doubles.
template <bool MIXED, int BPL, int WAVES>
__device__ __forceinline__ void process_tile(const Prepared& p, const float* __restrict__ acoef32, void* hp, void* hc,
                                             long k0, const Lds& L, double* red) {
  constexpr int TILE = 64 * BPL;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int Nf = p.Nf, nseg = p.K - 1;
  const long k1 = (k0 + TILE - 1 < Nf - 1) ? k0 + TILE - 1 : Nf - 1;

  double fk[BPL];
  Acc<MIXED> acc[BPL];
#pragma unroll
  for (int j = 0; j < BPL; ++j) {
    const long k = k0 + j * 64 + lane;
    fk[j] = (k < Nf) ? p.f[k] : 0.0;
    acc[j].zero();
  }

  // modes whose bin range meets the tile, 64 at a time, by ballot
  for (int mc = 0; mc < p.Nm; mc += 64) {
    const int mu = mc + lane;
    bool act = false;
    if (mu < p.Nm) {
      const int2 r = p.mode_kr[mu];
      act = (r.x <= k1) && (r.y >= k0);
    }
    unsigned long long mask = __ballot(act);
    while (mask) {
      const int bit = __ffsll((long long)mask) - 1;
      mask &= mask - 1;
      const int mode = mc + bit;
      const ModeConst md = p.modes[mode];
      const Piece* pcs = p.pieces + (size_t)mode * kMaxPieces;
      const double* ac = p.acoef + (size_t)mode * nseg * 8;
      const float* ac32 = MIXED ? acoef32 + (size_t)mode * nseg * 8 : nullptr;
      for (int q = 0; q < md.npieces; ++q) {
        const Piece P = pcs[q];
        if (P.k_lo > k1 || P.k_hi < k0) continue;
        if ((mode + q) % WAVES != wave) continue;
#pragma unroll
        for (int j = 0; j < BPL; ++j) {
          // bins of this piece in sub-tile j (wave-uniform)
          const long ka = max(k0 + j * 64, (long)P.k_lo);
          const long kz = min(min(k0 + j * 64 + 63, (long)Nf - 1), (long)P.k_hi);
          if (ka > kz) continue;
          const long k = k0 + j * 64 + lane;
          if (k >= ka && k <= kz)
            eval_bin<MIXED>(fk[j], P, md.m, md.n, md.cp_re, md.cp_im, md.cx_re, md.cx_im, ac, ac32, L, acc[j]);
        }
      }
    }
  }

  // partial sums of the waves, added in wave order
#pragma unroll
  for (int j = 0; j < BPL; ++j) {
    double* r = red + ((size_t)(wave * BPL + j) * 64 + lane) * 4;
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      if constexpr (MIXED)
        r[c] = (double)acc[j].v[c] - (double)acc[j].c[c];
      else
        r[c] = acc[j].v[c];
    }
  }
  __syncthreads();
  for (int t = threadIdx.x; t < TILE; t += 64 * WAVES) {
    const int j = t >> 6, ln = t & 63;
    const long k = k0 + t;
    double v[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int w = 0; w < WAVES; ++w) {
      const double* r = red + ((size_t)(w * BPL + j) * 64 + ln) * 4;
#pragma unroll
      for (int c = 0; c < 4; ++c) v[c] += r[c];
    }
    if (k < Nf) {
      if constexpr (MIXED) {
        ((float2*)hp)[k] = make_float2((float)v[0], (float)v[1]);
        ((float2*)hc)[k] = make_float2((float)v[2], (float)v[3]);
      } else {
        ((double2*)hp)[k] = make_double2(v[0], v[1]);
        ((double2*)hc)[k] = make_double2(v[2], v[3]);
      }
    }
  }
}

template <int BPL, int WAVES>
constexpr size_t red_doubles() {
  return (size_t)WAVES * BPL * 64 * 4;
}

template <bool MIXED, int BPL, int WAVES>
__global__ __launch_bounds__(64 * WAVES) void gather_kernel(GatherArgs a) {
  extern __shared__ double lds[];
  const Prepared& p = a.p;
  constexpr int TILE = 64 * BPL;
  const long k0 = (long)blockIdx.x * TILE;
  const long k1 = k0 + TILE - 1;
  // tiles outside the bin envelope of all modes only write zeros
  if (k1 < p.env[0] || k0 > p.env[1]) {
    zero_tile<MIXED, BPL, WAVES>(a.hp, a.hc, p.Nf, k0);
    return;
  }
  double* red = lds;
  const Lds L = stage_lds(p, lds + red_doubles<BPL, WAVES>());
  __syncthreads();
  process_tile<MIXED, BPL, WAVES>(p, a.acoef32, a.hp, a.hc, k0, L, red);
}

// Persistent gather over a batch: every workgroup repeatedly takes the next
// tile (waveform b, bins [j * 64 BPL, (j + 1) * 64 BPL)) from a device counter
// and evaluates it exactly as the single-waveform kernel would, restaging the
// LDS tables when the waveform changes.  The counter only schedules; every
// output element is computed in a fixed order, so results do not depend on
// the schedule.  Every workgroup leaves the loop once the counter passes the
// last tile.
template <bool MIXED, int BPL, int WAVES>
__global__ __launch_bounds__(64 * WAVES) void gather_batch_kernel(const WaveItem* __restrict__ items, int B,
                                                                  const int32_t* __restrict__ item_prefix,
                                                                  int total_items, int* __restrict__ counter) {
  extern __shared__ double lds[];
  __shared__ int s_item;
  constexpr int TILE = 64 * BPL;
  double* red = lds;
  double* tables = lds + red_doubles<BPL, WAVES>();
  int cached = -1;
  Lds L{};
  for (;;) {
    __syncthreads();
    if (threadIdx.x == 0) s_item = atomicAdd(counter, 1);
    __syncthreads();
    const int it = s_item;
    if (it >= total_items) break;
    int lo = 0, hi = B - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (item_prefix[mid] <= it)
        lo = mid;
      else
        hi = mid - 1;
    }
    const WaveItem& w = items[lo];
    const Prepared p = prepared_of(w);
    const long k0 = (long)(it - item_prefix[lo]) * TILE;
    const long k1 = k0 + TILE - 1;
    if (k1 < p.env[0] || k0 > p.env[1]) {
      zero_tile<MIXED, BPL, WAVES>(w.hp, w.hc, p.Nf, k0);
      continue;
    }
    if (lo != cached) {
      L = stage_lds(p, tables);
      __syncthreads();
      cached = lo;
    }
    process_tile<MIXED, BPL, WAVES>(p, w.acoef32, w.hp, w.hc, k0, L, red);
  }
}

__global__ void reset_counter_kernel(int* counter) { *counter = 0; }

// Normalised FP32 amplitude coefficients for the mixed path:
// A(t_i + u h) = sum_k (a_k h^k) u^k, u in [0, 1].
__global__ void amp32_kernel(int Nm, int K, const double* __restrict__ t, const double* __restrict__ acoef,
                             float* __restrict__ acoef32) {
  const int nseg = K - 1;
  const long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (long)Nm * nseg) return;
  const int i = (int)(idx % nseg);
  const double h = t[i + 1] - t[i];
  const double* c = acoef + idx * 8;
  float* o = acoef32 + idx * 8;
  double hk = 1.0;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    o[2 * k] = (float)(c[2 * k] * hk);
    o[2 * k + 1] = (float)(c[2 * k + 1] * hk);
    hk *= h;
  }
}

// Batched: one thread per (waveform, mode, segment) through the prefix of Nm_b (K_b - 1).
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
  const int idx = g - amp_prefix[lo];
  const int nseg = w.K - 1;
  const int i = idx % nseg;
  const double h = w.t[i + 1] - w.t[i];
  const double* c = w.acoef + (size_t)idx * 8;
  float* o = w.acoef32 + (size_t)idx * 8;
  double hk = 1.0;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    o[2 * k] = (float)(c[2 * k] * hk);
    o[2 * k + 1] = (float)(c[2 * k + 1] * hk);
    hk *= h;
  }
}

size_t gather_lds_bytes(int K) { return (size_t)(5 * K + 12 * (K - 1)) * sizeof(double); }

template <bool MIXED, int BPL, int WAVES>
static hipError_t launch_gather_t(const GatherArgs& a, hipStream_t stream) {
  constexpr int per_block = 64 * BPL;
  const long blocks = ((long)a.p.Nf + per_block - 1) / per_block;
  const size_t red = red_doubles<BPL, WAVES>() * sizeof(double);
  const size_t lds = gather_lds_bytes(a.p.K) + red;
  static bool attr_set = false;
  if (!attr_set) {
    (void)hipFuncSetAttribute((const void*)gather_kernel<MIXED, BPL, WAVES>, hipFuncAttributeMaxDynamicSharedMemorySize,
                              (int)(gather_lds_bytes(kMaxKnots) + red));
    attr_set = true;
  }
  gather_kernel<MIXED, BPL, WAVES><<<dim3((unsigned)blocks), dim3(64 * WAVES), lds, stream>>>(a);
  return hipGetLastError();
}

hipError_t launch_gather(const GatherArgs& a, bool mixed, int bpl, hipStream_t stream) {
  if (mixed) {
    if (bpl == 1) return launch_gather_t<true, 1, 4>(a, stream);
    if (bpl == 2) return launch_gather_t<true, 2, 4>(a, stream);
    return launch_gather_t<true, 4, 4>(a, stream);
  }
  if (bpl == 1) return launch_gather_t<false, 1, 4>(a, stream);
  if (bpl == 2) return launch_gather_t<false, 2, 4>(a, stream);
  return launch_gather_t<false, 4, 4>(a, stream);
}

hipError_t launch_gather_flat(const Prepared& p, const float* acoef32, void* hp, void* hc, bool mixed, int bpl,
                              hipStream_t stream) {
  GatherArgs a;
  a.p = p;
  a.acoef32 = acoef32;
  a.hp = hp;
  a.hc = hc;
  return launch_gather(a, mixed, bpl, stream);
}

template <bool MIXED, int BPL, int WAVES>
static hipError_t launch_gather_batch_t(const WaveItem* items, int B, const int32_t* item_prefix, int total_items,
                                        int* counter, int Kmax, int grid, hipStream_t stream) {
  const size_t red = red_doubles<BPL, WAVES>() * sizeof(double);
  const size_t lds = gather_lds_bytes(Kmax) + red;
  static bool attr_set = false;
  if (!attr_set) {
    (void)hipFuncSetAttribute((const void*)gather_batch_kernel<MIXED, BPL, WAVES>,
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)(gather_lds_bytes(kMaxKnots) + red));
    attr_set = true;
  }
  reset_counter_kernel<<<1, 1, 0, stream>>>(counter);
  gather_batch_kernel<MIXED, BPL, WAVES><<<dim3(grid), dim3(64 * WAVES), lds, stream>>>(items, B, item_prefix,
                                                                                     total_items, counter);
  return hipGetLastError();
}

// Number of workgroups of the persistent kernel: enough to fill every CU.
template <bool MIXED, int BPL, int WAVES>
static int persistent_grid(int Kmax) {
  int dev = 0, ncu = 0, per_cu = 0;
  (void)hipGetDevice(&dev);
  (void)hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
  (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void*)gather_batch_kernel<MIXED, BPL, WAVES>,
                                                     64 * WAVES,
                                                     gather_lds_bytes(Kmax) + red_doubles<BPL, WAVES>() * sizeof(double));
  if (ncu <= 0) ncu = 256;
  if (per_cu <= 0) per_cu = 1;
  return ncu * per_cu;
}

int gather_items_per_waveform(int Nf, int bpl) {
  const int per_tile = 64 * bpl;
  return (Nf + per_tile - 1) / per_tile;
}

hipError_t launch_gather_batch(const WaveItem* items, int B, const int32_t* item_prefix, int total_items,
                               int* counter, int Kmax, bool mixed, int bpl, hipStream_t stream) {
  if (mixed) {
    if (bpl == 1)
      return launch_gather_batch_t<true, 1, 4>(items, B, item_prefix, total_items, counter, Kmax,
                                               persistent_grid<true, 1, 4>(Kmax), stream);
    if (bpl == 2)
      return launch_gather_batch_t<true, 2, 4>(items, B, item_prefix, total_items, counter, Kmax,
                                               persistent_grid<true, 2, 4>(Kmax), stream);
    return launch_gather_batch_t<true, 4, 4>(items, B, item_prefix, total_items, counter, Kmax,
                                             persistent_grid<true, 4, 4>(Kmax), stream);
  }
  if (bpl == 1)
    return launch_gather_batch_t<false, 1, 4>(items, B, item_prefix, total_items, counter, Kmax,
                                              persistent_grid<false, 1, 4>(Kmax), stream);
  if (bpl == 2)
    return launch_gather_batch_t<false, 2, 4>(items, B, item_prefix, total_items, counter, Kmax,
                                              persistent_grid<false, 2, 4>(Kmax), stream);
  return launch_gather_batch_t<false, 4, 4>(items, B, item_prefix, total_items, counter, Kmax,
                                            persistent_grid<false, 4, 4>(Kmax), stream);
}

hipError_t launch_amp32_batch(const WaveItem* items, int B, const int32_t* amp_prefix, int total, hipStream_t stream) {
  const int threads = 256;
  amp32_batch_kernel<<<(total + threads - 1) / threads, threads, 0, stream>>>(items, B, amp_prefix, total);
  return hipGetLastError();
}

hipError_t launch_amp32(int Nm, int K, const double* t, const double* acoef, float* acoef32, hipStream_t stream) {
  const long total = (long)Nm * (K - 1);
  const int threads = 256;
  amp32_kernel<<<dim3((unsigned)((total + threads - 1) / threads)), threads, 0, stream>>>(Nm, K, t, acoef, acoef32);
  return hipGetLastError();
}

}  // namespace fdemri
