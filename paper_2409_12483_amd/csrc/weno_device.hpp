// 1-D polynomial WENO of degree NW (1, 2 or 3) from 2 NW + 1 cell averages
// to nodal values at the n = NW + 1 Gauss-Legendre nodes of the centre cell,
// with the tables of operators.cpp: degree 1 uses the stencils {i-1, i} and
// {i, i+1}, degree 2 {i-2..i}, {i-1..i+1}, {i..i+2}, degree 3 {i-3..i},
// {i-2..i+1}, {i-1..i+2}, {i..i+3}; weights lambda_s / (sigma_s + 1e-14)^8
// (lambda = 1e5 for the central stencils of degrees 2 and 3, else 1), the
// indicators sigma_s evaluated on differences from the centre value (their
// quadratic forms vanish on constants).  Shared by the 2-D and 3-D
// finite-volume kernels.
#pragma once

#include "device_common.hpp"

namespace aderdg {

template <int NW>
__device__ __forceinline__ void weno1d(const double (&v)[2 * NW + 1], const DevWeno& T, double* out,
                                       int k_only) {
  constexpr int n = NW + 1, NS = NW == 1 ? 2 : (NW % 2 ? 4 : 3);
  double wsum = 0.0, acc[n];
#pragma unroll
  for (int k = 0; k < n; ++k) acc[k] = 0.0;
#pragma unroll
  for (int s = 0; s < NS; ++s) {
    // first cell of the stencil, 0 = i - NW
    const int off = NW == 1 ? s
                  : NW % 2 ? (s == 0 ? 0 : s == 1 ? (NW - 1) / 2 : s == 2 ? (NW + 1) / 2 : NW)
                           : (s == 0 ? 0 : s == 1 ? NW / 2 : NW);
    const bool central = NW == 1 ? false : NW % 2 ? (s == 1 || s == 2) : s == 1;
    double d[n];
#pragma unroll
    for (int q = 0; q < n; ++q) d[q] = v[off + q] - v[NW];
    double sig = 0.0;
#pragma unroll
    for (int q = 0; q < n; ++q) {
      double si = 0.0;
#pragma unroll
      for (int m = 0; m < n; ++m) si += T.S[s][q][m] * d[m];
      sig += d[q] * si;
    }
    const double e = sig + 1.0e-14;
    const double e2 = e * e, e4 = e2 * e2, e8 = e4 * e4;
    const double om = (central ? 1.0e5 : 1.0) / e8;
    wsum += om;
#pragma unroll
    for (int k = 0; k < n; ++k) {
      if (k_only >= 0 && k != k_only) continue;
      double val = 0.0;
#pragma unroll
      for (int q = 0; q < n; ++q) val += T.R[s][k][q] * v[off + q];
      acc[k] += om * val;
    }
  }
#pragma unroll
  for (int k = 0; k < n; ++k) out[k] = acc[k] / wsum;
}

}  // namespace aderdg
