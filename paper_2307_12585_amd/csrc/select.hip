// Mode selection by power (Sec. 2.1: the waveform keeps the modes whose
// share of the total power is above a threshold; the share is taken at every
// knot of the trajectory and a mode is kept if it passes at one of them).
//
//   P_i = sum_mu |A_mu(t_i)|^2,   keep mu  <=>  |A_mu(t_i)|^2 > eps P_i for some i,
//
// with |A|^2 = re re + im im rounded term by term (no fused multiply-add), the
// sums over rows in a fixed order (strided per thread, then a tree), and the
// kept rows listed in table order.  Three small kernels; all deterministic.
#include "fdemri_internal.hpp"

namespace fdemri {

__device__ __forceinline__ double power_of(double2 a) {
#pragma clang fp contract(off)
  const double x = a.x * a.x;
  const double y = a.y * a.y;
  return x + y;
}

constexpr int kSelThreads = 256;

// One workgroup per knot: P[i].
__global__ __launch_bounds__(kSelThreads) void knot_power_kernel(int K, int Nm, const double2* __restrict__ A,
                                                                 double* __restrict__ P) {
  __shared__ double red[kSelThreads];
  const int i = blockIdx.x;
  double s = 0.0;
  for (int mu = threadIdx.x; mu < Nm; mu += kSelThreads) s += power_of(A[(size_t)mu * K + i]);
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = kSelThreads / 2; w >= 1; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) P[i] = red[0];
}

// One thread per row: keep[mu] = 1 if the row passes at some knot.
__global__ __launch_bounds__(kSelThreads) void keep_kernel(int K, int Nm, const double2* __restrict__ A,
                                                           const double* __restrict__ P, double eps,
                                                           int32_t* __restrict__ keep) {
  const int mu = (int)blockIdx.x * kSelThreads + (int)threadIdx.x;
  if (mu >= Nm) return;
  int k = 0;
  const double2* row = A + (size_t)mu * K;
  for (int i = 0; i < K && !k; ++i)
    if (power_of(row[i]) > eps * P[i]) k = 1;
  keep[mu] = k;
}

// One workgroup: the kept rows in table order, by block-wide prefix sums over
// chunks of kSelThreads rows.
__global__ __launch_bounds__(kSelThreads) void compact_kernel(int Nm, const int32_t* __restrict__ keep,
                                                              int32_t* __restrict__ idx, int32_t* __restrict__ n_keep) {
  __shared__ int pre[kSelThreads];
  int base = 0;
  for (int c0 = 0; c0 < Nm; c0 += kSelThreads) {
    const int mu = c0 + (int)threadIdx.x;
    const int k = (mu < Nm) ? keep[mu] : 0;
    pre[threadIdx.x] = k;
    __syncthreads();
    // inclusive scan (Hillis-Steele)
    for (int off = 1; off < kSelThreads; off <<= 1) {
      const int v = ((int)threadIdx.x >= off) ? pre[threadIdx.x - off] : 0;
      __syncthreads();
      pre[threadIdx.x] += v;
      __syncthreads();
    }
    if (k) idx[base + pre[threadIdx.x] - 1] = mu;
    base += pre[kSelThreads - 1];
    __syncthreads();
  }
  if (threadIdx.x == 0) *n_keep = base;
}

hipError_t launch_select_modes(int K, int Nm, const double* A, double eps, double* P, int32_t* keep, int32_t* idx,
                               int32_t* n_keep, hipStream_t stream) {
  if (Nm > 0) {
    knot_power_kernel<<<K, kSelThreads, 0, stream>>>(K, Nm, (const double2*)A, P);
    keep_kernel<<<(Nm + kSelThreads - 1) / kSelThreads, kSelThreads, 0, stream>>>(K, Nm, (const double2*)A, P, eps,
                                                                                 keep);
  }
  compact_kernel<<<1, kSelThreads, 0, stream>>>(Nm, keep, idx, n_keep);
  return hipGetLastError();
}

}  // namespace fdemri

namespace fdemri {

// Frequency band of a waveform's voices (Sec. 3.3: a downsampled grid spans
// only the band the signal occupies): the smallest and largest |F_V| over the
// ends of all monotonic pieces of all voices.  One workgroup; min and max are
// exact, so the result does not depend on the order.
__global__ __launch_bounds__(kSelThreads) void band_kernel(int Nm, const ModeConst* __restrict__ modes,
                                                           const Piece* __restrict__ pieces, double* __restrict__ band) {
  __shared__ double lo[kSelThreads], hi[kSelThreads];
  double a = __builtin_inf(), b = 0.0;
  for (int mu = threadIdx.x; mu < Nm; mu += kSelThreads) {
    const int np = modes[mu].npieces;
    for (int q = 0; q < np; ++q) {
      const Piece& P = pieces[(size_t)mu * kMaxPieces + q];
      a = fmin(a, fmin(P.g_a, P.g_b));
      b = fmax(b, fmax(P.g_a, P.g_b));
    }
  }
  lo[threadIdx.x] = a;
  hi[threadIdx.x] = b;
  __syncthreads();
  for (int w = kSelThreads / 2; w >= 1; w >>= 1) {
    if ((int)threadIdx.x < w) {
      lo[threadIdx.x] = fmin(lo[threadIdx.x], lo[threadIdx.x + w]);
      hi[threadIdx.x] = fmax(hi[threadIdx.x], hi[threadIdx.x + w]);
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    band[0] = (lo[0] == __builtin_inf()) ? 0.0 : fabs(lo[0]);  // +0 for a zero crossing
    band[1] = hi[0];
  }
}

hipError_t launch_band(int Nm, const ModeConst* modes, const Piece* pieces, double* band, hipStream_t stream) {
  band_kernel<<<1, kSelThreads, 0, stream>>>(Nm, modes, pieces, band);
  return hipGetLastError();
}

}  // namespace fdemri
