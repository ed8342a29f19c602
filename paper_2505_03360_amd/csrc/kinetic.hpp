// Per-cell kinetic quantities shared by the IMEX kernels: the Maxwellians of
// the penalised update (Sec. 4.4, eq. (4.24)) are evaluated in the epilogues
// of the collision and projection kernels, as products of per-axis Gaussians,
// from parameters one reduction kernel computes per cell.
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

// f^{n+1} at one velocity node from the Maxwellians m0 = M^n, m1 = M^{n+1}
// there (eq. (4.24) with P(h) = beta (M[h] - h)):
//   (eps (f - dt tr) + dt (Q - beta (M^n - f)) + beta dt M^{n+1}) / (eps + beta dt)
__device__ __forceinline__ double imex_combine(double beta, double q, double f, double tr, double eps, double dt,
                                               double m0, double m1) {
  const double den = eps + beta * dt;
  return (eps * (f - dt * tr) + dt * (q - beta * (m0 - f)) + beta * dt * m1) / den;
}

// A Maxwellian on the grid is a product of one Gaussian per axis:
// exp(-|v - u|^2 / 2T) = prod_a exp(-(v_a - u_a)^2 / 2T).  Table entry
// [mw][axis][j] = exp(-(v_j - u_axis)^2 / 2T) of Maxwellian mw (0: M^n, 1:
// M^{n+1}), v_j = (j - n/2) dv; 6 n doubles per cell.
__device__ __forceinline__ double axis_gaussian(const double* par, int mw, int axis, int j, int n, double dv) {
  const double d = (j - n / 2) * dv - par[5 * mw + 1 + axis];
  return exp(-d * d * par[5 * mw + 4]);
}

}  // namespace bzk
