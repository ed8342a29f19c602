// Per-cell kinetic quantities shared by the IMEX kernels: the Maxwellians of
// the penalised update (Sec. 4.4, eq. (4.24)) are evaluated pointwise in the
// epilogues of the collision kernels from parameters one reduction kernel
// computes per cell.
#pragma once

#include <hip/hip_runtime.h>

namespace bzk {

// Per-cell parameter record written by the reduction kernel (doubles):
//   [0] c0 = rho^n / (2 pi T^n)^(3/2)   [1..3] u^n   [4] 1 / (2 T^n)
//   [5] c1 = rho^{n+1} / (2 pi T^{n+1})^(3/2)  [6..8] u^{n+1}  [9] 1 / (2 T^{n+1})
//   [10] beta = 2 pi rho^{n+1}
constexpr int kImexPar = 12;

struct ImexDev {
  const double* par;        // [cell][kImexPar], by position in the batch
  const double* f;          // f^n, FP64, rows as the collision input
  const double* tr;         // v . grad_x f^n, FP64, same rows
  const double* eps_cells;  // Knudsen number per row, or null
  double eps;               // Knudsen number when eps_cells is null
  double dt;
};

// f^{n+1} at one velocity node (eq. (4.24) with P(h) = beta (M[h] - h)):
//   (eps (f - dt tr) + dt (Q - beta (M^n - f)) + beta dt M^{n+1}) / (eps + beta dt)
__device__ __forceinline__ double imex_point(const double* par, double q, double f, double tr, double eps,
                                             double dt, double v1, double v2, double v3) {
  const double d01 = v1 - par[1], d02 = v2 - par[2], d03 = v3 - par[3];
  const double d11 = v1 - par[6], d12 = v2 - par[7], d13 = v3 - par[8];
  const double m0 = par[0] * exp(-(d01 * d01 + d02 * d02 + d03 * d03) * par[4]);
  const double m1 = par[5] * exp(-(d11 * d11 + d12 * d12 + d13 * d13) * par[9]);
  const double beta = par[10];
  const double den = eps + beta * dt;
  return (eps * (f - dt * tr) + dt * (q - beta * (m0 - f)) + beta * dt * m1) / den;
}

}  // namespace bzk
