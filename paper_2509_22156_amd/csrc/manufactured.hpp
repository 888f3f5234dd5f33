// Manufactured-solution heat problem (Section 4.2): on [0,1]^d,
//   u*(x, t) = sqrt(|x|^2 + t^2) e^-t prod_i sin(pi x_i),
// and the forcing f = du*/dt - Laplace(u*) that makes u* exact. With
// r = sqrt(|x|^2 + t^2), S = prod_i sin(pi x_i), S_i = S without factor i:
//   du*/dt     = e^-t S (t/r - r)
//   Laplace u* = e^-t [S (d/r - |x|^2/r^3) + (2 pi/r) sum_i x_i cos(pi x_i) S_i
//                      - d pi^2 r S]
#pragma once

#include "line_layout.hpp"

namespace ctm {

constexpr double kPi = 3.14159265358979323846;

// f from the per-node pieces: S, C = sum_i x_i cos(pi x_i) S_i, |x|^2.
__device__ __forceinline__ double mms_f(double S, double C, double x2, int d, double t,
                                        double E) {
  const double r = sqrt(x2 + t * t);
  const double ir = 1.0 / r;
  const double dudt = S * (t * ir - r);
  const double lap = S * ((double)d * ir - x2 * ir * ir * ir) + 2.0 * kPi * ir * C -
                     (double)d * kPi * kPi * r * S;
  return E * (dudt - lap);
}

__device__ __forceinline__ double mms_exact(const double* x, int d, double t) {
  double x2 = 0.0, S = 1.0;
  for (int i = 0; i < d; ++i) {
    x2 += x[i] * x[i];
    S *= sinpi(x[i]);
  }
  return sqrt(x2 + t * t) * exp(-t) * S;
}

// f(., t) at the unknowns of the lane's chunk (zero in padding slots). The
// products over the non-stiff axes are built once, then extended by the
// stiff coordinate of each unknown.
template <int K>
__device__ __forceinline__ void mms_forcing(const GridDev& g, const Lane<K>& L, double t,
                                            double (&f)[K]) {
  double P = 1.0, C = 0.0, X2 = 0.0;
#pragma unroll
  for (int m = 0; m < MAXD - 1; ++m) {
    if (m < g.d - 1) {
      const int ax = g.oax[m];
      const double x = g.lo[ax] + (double)(L.jo[m] + g.j0) * g.h[ax];
      double sn, cs;
      sincospi(x, &sn, &cs);
      C = C * sn + x * cs * P;
      P *= sn;
      X2 += x * x;
    }
  }
  const int s = g.sax;
  const double E = exp(-t);
#pragma unroll
  for (int k = 0; k < K; ++k) {
    f[k] = 0.0;
    if (k < L.nval) {
      const double x = g.lo[s] + (double)(L.j0 + k + g.j0) * g.h[s];
      double sn, cs;
      sincospi(x, &sn, &cs);
      f[k] = mms_f(P * sn, C * sn + x * cs * P, X2 + x * x, g.d, t, E);
    }
  }
}

// f(x_p, t) at canonical point p of grid g (axis d-1 fastest), for the
// streaming solvers, which sweep points rather than lanes' chunks.
template <int D>
__device__ __forceinline__ double mms_point(const GridDev& g, int p, double t) {
  double P = 1.0, C = 0.0, X2 = 0.0;
  int rem = p;
#pragma unroll
  for (int i = D - 1; i >= 0; --i) {
    if (i < g.d) {
      const int j = rem % g.n[i];
      rem /= g.n[i];
      const double x = g.lo[i] + (double)(j + g.j0) * g.h[i];
      double sn, cs;
      sincospi(x, &sn, &cs);
      C = C * sn + x * cs * P;
      P *= sn;
      X2 += x * x;
    }
  }
  return mms_f(P, C, X2, g.d, t, exp(-t));
}

}  // namespace ctm
