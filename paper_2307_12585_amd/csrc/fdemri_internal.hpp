// Internal structures and device helpers of the frequency-domain EMRI mode
// sum (Sec. 2.2 of arXiv 2307.12585).  Shared by the kernels of this
// library only.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/fdemri.h"

namespace fdemri {

constexpr int kMaxPieces = FDEMRI_MAX_PIECES;
constexpr int kMaxKnots = FDEMRI_MAX_KNOTS;
constexpr int kMaxL = FDEMRI_MAX_L;

// 2 pi as an unevaluated double-double (2 pi = kTwoPiHi + kTwoPiLo to ~1e-32).
constexpr double kTwoPiHi = 6.283185307179586232e+00;
constexpr double kTwoPiLo = 2.449293598294706414e-16;
constexpr double kInvTwoPi = 0.15915494309189535;
constexpr double kPi = 3.141592653589793116;

// One monotonic piece of a voice frequency F_V(t) = m F_phi + n F_r over the
// sparse trajectory: F_V has one sign s on it and |F_V| is monotonic with
// direction d in t.  It starts at tau_a inside spline segment seg_a and ends
// at tau_b inside segment seg_b; g_a, g_b are |F_V| at the two ends, and
// [k_lo, k_hi] the bins whose frequency lies in [min, max](g_a, g_b).
// rate f + rate0, with rate = (seg_b - seg_a + 1) / (g_b - g_a) and
// rate0 = seg_a - rate g_a, gives a first guess of the segment holding a
// frequency f (the search that follows does not depend on it); dd and sd are
// d and s as doubles.  whole = 1 when the piece runs from the first knot of the
// trajectory to the last (no turning point or zero crossing): then its end
// values are the knot values, bit for bit.
struct alignas(32) Piece {
  double tau_a, tau_b;
  double g_a, g_b;
  double rate, rate0;
  double dd, sd;
  int32_t seg_a, seg_b;
  int32_t k_lo, k_hi;
  int32_t s, d;
  int32_t whole, pad;
};
static_assert(sizeof(Piece) == 96, "Piece layout");

// Per-mode constants: mode numbers as doubles and the fused polarization
// factors c_+ and c_x (scale and spin-weighted harmonics folded in).
struct alignas(64) ModeConst {
  double m, n;
  double cp_re, cp_im, cx_re, cx_im;
  int32_t npieces, pad;
  int32_t k_lo, k_hi;
};
static_assert(sizeof(ModeConst) == 64, "ModeConst layout");

// Voice-frequency groups.  Rows with the same (m, n) have the same voice
// frequency F_V = m F_phi + n F_r, hence the same monotonic pieces, roots,
// phases and factors G; only the amplitude A_lmn and the harmonics in c_+,
// c_x differ.  The set-up sorts the rows by (m, n) (then by row index) into
// groups; the gather solves each root once per group and adds every member's
// amplitude term.  A member: its row and its fused polarization factors.
struct alignas(16) GroupMember {
  double cp_re, cp_im, cx_re, cx_im;
  int32_t mode, pad[3];
};
static_assert(sizeof(GroupMember) == 48, "GroupMember layout");
struct alignas(16) GroupMember32 {
  float4 c;  // (c_+, c_x) in FP32
  int32_t mode, pad[3];
};
static_assert(sizeof(GroupMember32) == 32, "GroupMember32 layout");

// Mode tables above this size get a bin envelope (a launch after the set-up;
// a smaller table is scanned by the gather as cheaply as the launch would
// cost) and, up to kGroupMaxModes rows (the keys the set-up's sort holds
// in registers), voice groups.
constexpr int kEnvelopeMinModes = 256;
constexpr int kGroupMaxModes = 4096;
__host__ __device__ inline bool modes_grouped(int Nm) { return Nm > kEnvelopeMinModes && Nm <= kGroupMaxModes; }

// FP32 coefficients of one amplitude segment (8 doubles: re, im of the powers
// 0..3 of tau) in the normalised variable u = tau / h, as the mixed path
// reads them: A(t_i + u h) = sum_k (a_k h^k) u^k, u in [0, 1].
__device__ __forceinline__ void amp32_segment(const double* __restrict__ c, double h, float* __restrict__ o) {
  const double h2 = h * h, h3 = h2 * h;
  o[0] = (float)c[0];
  o[1] = (float)c[1];
  o[2] = (float)(c[2] * h);
  o[3] = (float)(c[3] * h);
  o[4] = (float)(c[4] * h2);
  o[5] = (float)(c[5] * h2);
  o[6] = (float)(c[6] * h3);
  o[7] = (float)(c[7] * h3);
}

// Device pointers of one waveform's prepared tables.
struct Prepared {
  int32_t K, Nm, Nf;
  const double* t;       // [K]
  const double* Fphi;    // [K]
  const double* Fr;      // [K]
  const double* Phiphi;  // [K]
  const double* Phir;    // [K]
  const double* f;       // [Nf]
  const double* tcoef;   // [4][K-1][4] Fphi, Fr, Phiphi, Phir; ascending powers
  const double* acoef;   // [Nm][K-1][8] amplitude (re,im) x ascending powers
  const ModeConst* modes;  // [Nm]
  const int2* mode_kr;     // [Nm] bin range of each mode (union of its pieces)
  const Piece* pieces;     // [Nm][kMaxPieces]
  const int32_t* status;   // [3] input status of the call (0: valid; see the input checks below),
                           // then the bin envelope [lo, hi] of all voices (the whole grid unless formed)
  const float4* modes32;   // [Nm] (c_+, c_x) of each mode in FP32 (mixed path only)
  // voice groups (all NULL when the rows are not grouped): per position of
  // the sorted rows, the group's bin range at its first position (empty
  // elsewhere), the group size there (0 elsewhere), and the member
  const int2* gkr;
  const int32_t* gsize;
  const GroupMember* gmem;
  const GroupMember32* gmem32;  // mixed path
  const int32_t* slots;    // [nslots] input status per check workgroup, when the set-up was fused
  int32_t nslots;          // (then status is not read and the envelope is the whole grid); 0 otherwise
};

// Device-resident record of one waveform of a batch: caller inputs, the
// library's scratch tables for it, and its outputs.
struct WaveItem {
  int32_t K, Nm, Nf;
  uint32_t flags;
  const double *t, *Fphi, *Fr, *Phiphi, *Phir, *A, *f;
  const int32_t *l, *m, *n;
  double theta, phi, scale;
  double* tcoef;
  double* acoef;
  float* acoef32;
  ModeConst* modes;
  float4* modes32;  // mixed path: (c_+, c_x) in FP32
  int2* mode_kr;
  Piece* pieces;
  int64_t* evals;
  int32_t* status;  // [3] input status of the waveform, bin envelope [lo, hi]
  int2* gkr;        // voice groups (NULL unless modes_grouped(Nm))
  int32_t* gsize;
  GroupMember* gmem;
  GroupMember32* gmem32;
  void* hp;
  void* hc;
  // fused likelihood of the batch: data, per-bin weights and this waveform's
  // partial-sum and edge-record scratch (unused for a waveform batch)
  const void* d_p;
  const void* d_c;
  const double* wS;
  double* ll_partial;
  double* ll_edge;
};

__host__ __device__ inline Prepared prepared_of(const WaveItem& w) {
  Prepared p;
  p.K = w.K;
  p.Nm = w.Nm;
  p.Nf = w.Nf;
  p.t = w.t;
  p.Fphi = w.Fphi;
  p.Fr = w.Fr;
  p.Phiphi = w.Phiphi;
  p.Phir = w.Phir;
  p.f = w.f;
  p.tcoef = w.tcoef;
  p.acoef = w.acoef;
  p.modes = w.modes;
  p.mode_kr = w.mode_kr;
  p.pieces = w.pieces;
  p.status = w.status;
  p.modes32 = w.modes32;
  p.gkr = w.gkr;
  p.gsize = w.gsize;
  p.gmem = w.gmem;
  p.gmem32 = w.gmem32;
  p.slots = nullptr;
  p.nslots = 0;
  return p;
}

// Input checks on the device (the host does not read device data): a
// waveform whose inputs fail them has status bits in its status word, every
// kernel writes zeros for it, and FDEMRI_FLAG_BAD_INPUT is raised.  The first
// launch of a call clears the status; workgroups of the set-up launch run the
// checks; the gather and the adjoint read it.
constexpr int32_t kBadKnots = 1;     // t not finite or not strictly increasing
constexpr int32_t kBadValues = 2;    // a trajectory or amplitude value not finite
constexpr int32_t kBadGrid = 4;      // f not finite, negative or descending
constexpr int32_t kBadHannGrid = 8;  // Hann kernel asked for on a grid that is not k f_1
// Elements checked per workgroup of the checks.
constexpr int kCheckChunk = 4096;

// Fused set-up of small waveforms (one launch for the trajectory splines, the
// piece tables, the amplitude splines and the checks): at most this many
// modes (the tables the gather scans without an envelope), knots and check
// workgroups, whose statuses then go to one slot each instead of a status
// word that an earlier launch would have to clear.
constexpr int kFusedMaxModes = 256;
constexpr int kFusedMaxKnots = 256;
constexpr int kFusedMaxSlots = 256;

// Workgroups of the checks of one waveform: the trajectory, the amplitude
// array (knot values or given coefficients), the frequency grid.
__host__ __device__ inline long check_amp_count(int K, int Nm, uint32_t flags) {
  return (flags & FDEMRI_COEFFS_GIVEN) ? (long)Nm * (K - 1) * 8 : (long)Nm * K * 2;
}
__host__ __device__ inline int check_blocks(int K, int Nm, int Nf, uint32_t flags) {
  return 1 + (int)((check_amp_count(K, Nm, flags) + kCheckChunk - 1) / kCheckChunk) +
         (int)(((long)Nf + kCheckChunk - 1) / kCheckChunk);
}

// Qualifier of read-only device tables read through the constant address
// space (wave-uniform loads from it become scalar loads).  The host pass,
// which only checks device code, has no such address space.
#if defined(__HIP_DEVICE_COMPILE__)
#define kconst __attribute__((address_space(4)))
#else
#define kconst
#endif

// ---------------------------------------------------------------- helpers

struct dd {
  double hi, lo;
};

__device__ __forceinline__ dd two_prod(double a, double b) {
  double p = a * b;
  return {p, __builtin_fma(a, b, -p)};
}

__device__ __forceinline__ dd two_sum(double a, double b) {
#pragma clang fp contract(off)
  double s = a + b;
  double bb = s - a;
  double e = (a - (s - bb)) + (b - bb);
  return {s, e};
}

// Voice frequency at a knot from the knot data, with a fixed operation order
// and no fused multiply-add, so that every implementation of the piece
// boundaries agrees bit for bit.
__device__ __forceinline__ double knot_freq(double m, double fphi, double n, double fr) {
#pragma clang fp contract(off)
  double a = m * fphi;
  double b = n * fr;
  return a + b;
}

// m x + n y with one fused multiply-add in a fixed order, so that the
// forward and adjoint kernels form identical mode-weighted coefficients.
__device__ __forceinline__ double wsum(double m, double x, double n, double y) { return __builtin_fma(m, x, n * y); }

// a b + c for a constant c, as one three-operand FP64 fused multiply-add
// reading c from a scalar register pair.  Written out because the compiler
// otherwise keeps such constants in vector registers, hoisted out of the
// loops, and copies one into the destination before every two-operand
// multiply-add of a Horner step: an extra vector instruction per step and
// two vector registers held per constant.
__device__ __forceinline__ double fma_sc(double a, double b, double c) {
#if defined(__HIP_DEVICE_COMPILE__)
  double r;
  asm("v_fma_f64 %0, %1, %2, %3" : "=v"(r) : "v"(a), "v"(b), "s"(c));
  return r;
#else
  return __builtin_fma(a, b, c);
#endif
}

// x converted to int32 with the hardware's saturating conversion (out-of-range
// values go to the nearest end of the range, NaN to 0), without the undefined
// behaviour of a C++ conversion of such values.
__device__ __forceinline__ int cvt_i32_sat(double x) {
#if defined(__HIP_DEVICE_COMPILE__)
  int r;
  asm("v_cvt_i32_f64 %0, %1" : "=v"(r) : "v"(x));
  return r;
#else
  return (int)x;
#endif
}

// Reciprocal and reciprocal square root from the hardware estimates refined
// by Newton-Raphson steps (one step: for iterations that correct themselves;
// two steps: full double precision).
__device__ __forceinline__ double rcp_nr1(double x) {
  const double y = __builtin_amdgcn_rcp(x);
  return __builtin_fma(y, __builtin_fma(-x, y, 1.0), y);
}

__device__ __forceinline__ double rcp_nr2(double x) {
  double y = __builtin_amdgcn_rcp(x);
  y = __builtin_fma(y, __builtin_fma(-x, y, 1.0), y);
  return __builtin_fma(y, __builtin_fma(-x, y, 1.0), y);
}

__device__ __forceinline__ double rsq_nr2(double x) {
  double y = __builtin_amdgcn_rsq(x);
  y = __builtin_fma(0.5 * y, __builtin_fma(-x * y, y, 1.0), y);
  return __builtin_fma(0.5 * y, __builtin_fma(-x * y, y, 1.0), y);
}

}  // namespace fdemri
