// Searches in an ascending frequency array f[0..Nf) (the grid of the
// frequency-domain sum).  Bin ranges of pieces and segments are found by
// these, so their cost is a chain of dependent global loads: the first probe
// is a linear-interpolation guess between the bracket ends, checked together
// with its right neighbour in one round trip (exact on a uniform grid), and
// the search then alternates interpolation and bisection steps, so that any
// ascending grid is resolved in at most about 2 log2(Nf) probes.
#pragma once

#include "fdemri_internal.hpp"

namespace fdemri {

// First index k in [0, Nf] with f[k] >= x (strict = false) or f[k] > x
// (strict = true).
template <bool STRICT>
__device__ __forceinline__ int first_index(const double* __restrict__ f, int Nf, double x) {
  if (Nf <= 0) return 0;
  auto before = [&](double v) { return STRICT ? !(v > x) : (v < x); };  // v precedes the answer
  double fa = f[0], fb = f[Nf - 1];
  if (!before(fa)) return 0;
  if (before(fb)) return Nf;
  // invariant: before(f[a]) and !before(f[b]); the answer lies in (a, b]
  int a = 0, b = Nf - 1;
  bool interp = true;
  while (b - a > 1) {
    int g;
    if (interp && fb > fa) {
      const double u = (x - fa) / (fb - fa) * (double)(b - a);
      g = a + (int)fmin(fmax(u, 0.0), (double)(b - a));
      g = min(max(g, a + 1), b - 1);
      // probe g and g + 1 together: on a uniform grid one of them ends the search
      const double v0 = f[g];
      const double v1 = (g + 1 < b) ? f[g + 1] : fb;
      if (!before(v0)) {
        b = g;
        fb = v0;
      } else if (before(v1)) {
        a = g + 1;
        fa = v1;
      } else {
        return g + 1;
      }
    } else {
      g = a + ((b - a) >> 1);
      const double v = f[g];
      if (before(v)) {
        a = g;
        fa = v;
      } else {
        b = g;
        fb = v;
      }
    }
    interp = !interp;
  }
  return b;
}

__device__ __forceinline__ int first_ge(const double* __restrict__ f, int Nf, double x) {
  return first_index<false>(f, Nf, x);
}

__device__ __forceinline__ int first_gt(const double* __restrict__ f, int Nf, double x) {
  return first_index<true>(f, Nf, x);
}

}  // namespace fdemri
