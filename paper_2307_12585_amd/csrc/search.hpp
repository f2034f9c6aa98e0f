// Searches in an ascending frequency array f[0..Nf) (the grid of the
// frequency-domain sum).  Bin ranges of pieces and segments are found by
// these, so their cost is a chain of dependent global loads.  Each
// interpolation round probes, in one round trip, the index that linear
// interpolation between the bracket ends predicts and, when both ends are
// positive, the index that interpolation in log f predicts (FP32 logarithms:
// only a guess, the probes decide), each with its right neighbour: on a
// uniform grid the first, on a logarithmic grid the second ends the search.
// Rounds alternate with bisection steps, so that any ascending grid is
// resolved in at most about 2 log2(Nf) round trips.
#pragma once

#include "fdemri_internal.hpp"

namespace fdemri {

// Index in (a, b) that interpolation predicts for y(x) between y(f[a]) = ya
// and y(f[b]) = yb.
__device__ __forceinline__ int interp_index(int a, int b, double ya, double yb, double yx) {
  const double u = (yx - ya) / (yb - ya) * (double)(b - a);
  const int g = a + (int)fmin(fmax(u, 0.0), (double)(b - a));
  return min(max(g, a + 1), b - 1);
}

// First index k in [0, Nf] with f[k] >= x (strict = false) or f[k] > x
// (strict = true), given the end values f0 = f[0] and fN = f[Nf - 1] (Nf >= 1;
// a caller with several searches loads them once).  Invariant: f[a] precedes
// the answer, f[b] does not; a probe at index g with value v narrows (a, b]
// whatever the order of probes.
template <bool STRICT>
__device__ __forceinline__ int first_index(const double* __restrict__ f, int Nf, double x, double f0, double fN) {
#define FDEMRI_BEFORE(v) (STRICT ? !((v) > x) : ((v) < x))
#define FDEMRI_PROBE(g, v)      \
  if (FDEMRI_BEFORE(v)) {       \
    if ((g) > a) {              \
      a = (g);                  \
      fa = (v);                 \
    }                           \
  } else if ((g) < b) {         \
    b = (g);                    \
    fb = (v);                   \
  }
  double fa = f0, fb = fN;
  if (!FDEMRI_BEFORE(fa)) return 0;
  if (FDEMRI_BEFORE(fb)) return Nf;
  int a = 0, b = Nf - 1;
  bool interp = true;
  while (b - a > 1) {
    if (interp && fb > fa) {
      const int b0 = b;
      const int g = interp_index(a, b, fa, fb, x);
      const double v0 = f[g];
      const double v1 = (g + 1 < b0) ? f[g + 1] : fb;
      if (fa > 0.0 && x > 0.0) {
        // the log-interpolated pair too, in the same round trip
        const int g2 = interp_index(a, b, __log2f((float)fa), __log2f((float)fb), __log2f((float)x));
        const double w0 = f[g2];
        const double w1 = (g2 + 1 < b0) ? f[g2 + 1] : fb;
        FDEMRI_PROBE(g2, w0)
        if (g2 + 1 < b0) {
          FDEMRI_PROBE(g2 + 1, w1)
        }
      }
      FDEMRI_PROBE(g, v0)
      if (g + 1 < b0) {
        FDEMRI_PROBE(g + 1, v1)
      }
    } else {
      const int g = a + ((b - a) >> 1);
      const double v = f[g];
      FDEMRI_PROBE(g, v)
    }
    interp = !interp;
  }
#undef FDEMRI_PROBE
#undef FDEMRI_BEFORE
  return b;
}

__device__ __forceinline__ int first_ge(const double* __restrict__ f, int Nf, double x, double f0, double fN) {
  return first_index<false>(f, Nf, x, f0, fN);
}

__device__ __forceinline__ int first_gt(const double* __restrict__ f, int Nf, double x, double f0, double fN) {
  return first_index<true>(f, Nf, x, f0, fN);
}

__device__ __forceinline__ int first_ge(const double* __restrict__ f, int Nf, double x) {
  return Nf <= 0 ? 0 : first_ge(f, Nf, x, f[0], f[Nf - 1]);
}

__device__ __forceinline__ int first_gt(const double* __restrict__ f, int Nf, double x) {
  return Nf <= 0 ? 0 : first_gt(f, Nf, x, f[0], f[Nf - 1]);
}

}  // namespace fdemri
