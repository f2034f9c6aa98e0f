// Element-wise evaluation of the per-root factor G of Eq. extendedspa1 by
// the same device code the mode sum runs at every root (spa.hpp), for n
// pairs of local derivatives.  Like the gather, each wavefront chooses the
// length of the large-argument series from the largest |1/X| among its 64
// lanes, so 64 consecutive elements share one choice.
#include "spa.hpp"

namespace fdemri {

template <bool MIXED>
__global__ __launch_bounds__(256) void spa_factor_kernel(int n, const double* __restrict__ gd,
                                                         const double* __restrict__ gdd,
                                                         const int32_t* __restrict__ dir, void* __restrict__ out) {
  const long i = (long)blockIdx.x * 256 + threadIdx.x;
  const bool in = i < n;
  // lanes past the end take W = 1 (gdd = 0), which leaves the wave's series
  // length to the elements
  const double a = in ? gd[i] : 1.0, b = in ? gdd[i] : 0.0;
  const int d = in ? dir[i] : 1;
  if constexpr (MIXED) {
    const float2 g = spa_factor32(a, b, d);
    if (in) ((float2*)out)[i] = g;
  } else {
    const double2 g = spa_factor64(a, b, d);
    if (in) ((double2*)out)[i] = g;
  }
}

hipError_t launch_spa_factor(int n, const double* gd, const double* gdd, const int32_t* dir, void* out, bool mixed,
                             hipStream_t stream) {
  if (n <= 0) return hipSuccess;
  const unsigned blocks = (unsigned)((n + 255) / 256);
  if (mixed)
    spa_factor_kernel<true><<<blocks, 256, 0, stream>>>(n, gd, gdd, dir, out);
  else
    spa_factor_kernel<false><<<blocks, 256, 0, stream>>>(n, gd, gdd, dir, out);
  return hipGetLastError();
}

}  // namespace fdemri
