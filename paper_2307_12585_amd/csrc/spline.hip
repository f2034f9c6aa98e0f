// Kernels and launchers of the not-a-knot cubic splines (Sec. 2.1, Sec. 2.2);
// the solve itself is in spline_core.hpp.
#include <climits>

#include "spline_core.hpp"

namespace fdemri {

template <int NT>
__global__ __launch_bounds__(NT) void spline_pcr_kernel(int K, const double* __restrict__ t,
                                                        const double* __restrict__ y0, const double* __restrict__ y1,
                                                        const double* __restrict__ y2, const double* __restrict__ y3,
                                                        const double* __restrict__ A, int n_series,
                                                        double* __restrict__ tcoef, double* __restrict__ acoef,
                                                        double* fac, int32_t* __restrict__ status) {
  __shared__ SplineLds<NT> S;
  // this call's input status starts clear (the checks run in a later
  // launch), and its bin envelope covers every bin unless a later launch
  // forms it
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    status[0] = 0;
    status[1] = 0;
    status[2] = INT_MAX;
  }
  // the first workgroup also records the reduction factors of the knot matrix
  spline_block<NT>(S, (int)blockIdx.x * kSeriesPerBlock, n_series, K, t, y0, y1, y2, y3, A, tcoef, acoef,
                   blockIdx.x == 0 ? fac : nullptr);
}

// Batched: block -> (waveform, group of series) through block_prefix (per
// waveform ceil((4 + Nm_b) / kSeriesPerBlock) blocks).
template <int NT>
__global__ __launch_bounds__(NT) void spline_batch_kernel(const WaveItem* __restrict__ items, int B,
                                                          const int32_t* __restrict__ block_prefix) {
  __shared__ SplineLds<NT> S;
  const int g = blockIdx.x;
  int lo = 0, hi = B - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (block_prefix[mid] <= g)
      lo = mid;
    else
      hi = mid - 1;
  }
  const WaveItem& w = items[lo];
  if (g == block_prefix[lo] && threadIdx.x == 0) w.status[0] = 0;  // the waveform's input status starts clear
  const int n_series = 4 + ((w.flags & FDEMRI_COEFFS_GIVEN) ? 0 : w.Nm);
  spline_block<NT>(S, (g - block_prefix[lo]) * kSeriesPerBlock, n_series, w.K, w.t, w.Fphi, w.Fr, w.Phiphi, w.Phir,
                   w.A, w.tcoef, w.acoef, nullptr, w.acoef32);
}

int spline_blocks(int n_series) { return (n_series + kSeriesPerBlock - 1) / kSeriesPerBlock; }

// Host launcher: coefficients of the four trajectory series and of Nm
// complex amplitude series, all on knots t[K], with NT = 256 threads per
// workgroup for K <= 256 and 512 above; when fac is not null, the reduction
// factors of the knot matrix are written to it (pcr_factor_doubles<NT>());
// the call's input status word is cleared and its bin envelope set to the
// whole grid.
hipError_t launch_spline(int K, const double* t, const double* Fphi, const double* Fr, const double* Phiphi,
                         const double* Phir, const double* A, int Nm, double* tcoef, double* acoef, double* fac,
                         int32_t* status, hipStream_t stream) {
  const int n_series = 4 + Nm;
  const dim3 grid(spline_blocks(n_series));
  if (K <= 256)
    spline_pcr_kernel<256><<<grid, 256, 0, stream>>>(K, t, Fphi, Fr, Phiphi, Phir, A, n_series, tcoef, acoef, fac, status);
  else
    spline_pcr_kernel<512><<<grid, 512, 0, stream>>>(K, t, Fphi, Fr, Phiphi, Phir, A, n_series, tcoef, acoef, fac, status);
  return hipGetLastError();
}

// Doubles of the factor table written by launch_spline for K knots.
size_t spline_factor_doubles(int K) {
  return K <= 256 ? (size_t)pcr_factor_doubles<256>() : (size_t)pcr_factor_doubles<512>();
}

hipError_t launch_spline_batch(const WaveItem* items, int B, const int32_t* block_prefix, int total_blocks, int Kmax,
                               hipStream_t stream) {
  dim3 grid(total_blocks);
  if (Kmax <= 64)
    spline_batch_kernel<64><<<grid, 64, 0, stream>>>(items, B, block_prefix);
  else if (Kmax <= 128)
    spline_batch_kernel<128><<<grid, 128, 0, stream>>>(items, B, block_prefix);
  else if (Kmax <= 256)
    spline_batch_kernel<256><<<grid, 256, 0, stream>>>(items, B, block_prefix);
  else
    spline_batch_kernel<512><<<grid, 512, 0, stream>>>(items, B, block_prefix);
  return hipGetLastError();
}

}  // namespace fdemri
