"""FP64 oracle of the per-cell kinetic quantities around the collision
operator: macroscopic fields, the Maxwellian, the L1 distance of the
kinetic-to-fluid criterion, and the penalised first-order IMEX update of the
Boltzmann layer.

TEST INFRASTRUCTURE ONLY (see package doc).

Grid: v_j = (j - N/2) dv, dv = 2L/N, j in [0,N)^3 (Sec. 4.1); integrals over
velocity are the grid sums times dv^3.

  moments      rho = int f, u = int v f / rho, T = int |v - u|^2 f / (3 rho)
               (Sec. 2, the fields that define the equilibria (H3)).
  maxwellian   M(v) = rho (2 pi T)^(-3/2) exp(-|v - u|^2 / (2 T)) (Sec. 2).
  l1_distance  || f - M[f] ||_{L1_v}, the quantity compared with delta_0 in
               the kinetic-to-fluid criterion (Sec. 3.3).
  imex_euler   the penalised scheme of Sec. 4.4 (eq. 1002): with the transport
               term tr = v . grad_x f^n given,
                 g = f^n - dt tr,  U^{n+1} = int phi g (phi = 1, v, |v|^2),
                 beta = 2 pi rho^{n+1},  P(h) = beta (M[h] - h),
                 f^{n+1} = eps/(eps + beta dt) g
                           + dt (Q(f^n) - P(f^n)) / (eps + beta dt)
                           + beta dt/(eps + beta dt) M^{n+1},
               M^{n+1} the Maxwellian of U^{n+1}.
"""
from __future__ import annotations

import math

import numpy as np

from . import spectral


def _grid(n: int, L: float):
    v = spectral.velocity_nodes(n, L)
    V1, V2, V3 = np.meshgrid(v, v, v, indexing="ij")
    return V1, V2, V3, (2.0 * L / n) ** 3


def moments(f: np.ndarray, n: int, L: float):
    """(rho, u[3], T) of one cell from the defining integrals (Sec. 2),
    the temperature from the centred second moment."""
    V1, V2, V3, w = _grid(n, L)
    rho = w * f.sum()
    u = np.array([w * (V1 * f).sum(), w * (V2 * f).sum(), w * (V3 * f).sum()]) / rho
    c2 = (V1 - u[0]) ** 2 + (V2 - u[1]) ** 2 + (V3 - u[2]) ** 2
    T = w * (c2 * f).sum() / (3.0 * rho)
    return rho, u, T


def maxwellian(rho: float, u, T: float, n: int, L: float) -> np.ndarray:
    V1, V2, V3, _ = _grid(n, L)
    c2 = (V1 - u[0]) ** 2 + (V2 - u[1]) ** 2 + (V3 - u[2]) ** 2
    return rho / (2.0 * math.pi * T) ** 1.5 * np.exp(-c2 / (2.0 * T))


def l1_distance(f: np.ndarray, n: int, L: float) -> float:
    """|| f - M[f] ||_{L1_v} with M[f] the Maxwellian of f's own moments."""
    rho, u, T = moments(f, n, L)
    w = (2.0 * L / n) ** 3
    return float(w * np.abs(f - maxwellian(rho, u, T, n, L)).sum())


def conserved(h: np.ndarray, n: int, L: float):
    """U = int (1, v, |v|^2) h, the collision invariants' moments."""
    V1, V2, V3, w = _grid(n, L)
    return np.array([w * h.sum(), w * (V1 * h).sum(), w * (V2 * h).sum(), w * (V3 * h).sum(),
                     w * ((V1 * V1 + V2 * V2 + V3 * V3) * h).sum()])


def maxwellian_of_conserved(U, n: int, L: float) -> tuple[np.ndarray, float]:
    """Maxwellian whose (rho, rho u, int |v|^2) are U; also returns rho."""
    rho = U[0]
    u = U[1:4] / rho
    T = (U[4] / rho - (u[0] * u[0] + u[1] * u[1] + u[2] * u[2])) / 3.0
    return maxwellian(rho, u, T, n, L), rho


def imex_combine(f: np.ndarray, tr: np.ndarray, q: np.ndarray, dt: float, eps: float, L: float) -> np.ndarray:
    """The update of eq. 1002 given Q(f^n) (any array q) and the transport term."""
    n = f.shape[0]
    g = f - dt * tr
    M1, rho1 = maxwellian_of_conserved(conserved(g, n, L), n, L)
    beta = 2.0 * math.pi * rho1
    rho0, u0, T0 = moments(f, n, L)
    P0 = beta * (maxwellian(rho0, u0, T0, n, L) - f)
    den = eps + beta * dt
    return (eps / den) * g + (dt / den) * (q - P0) + (beta * dt / den) * M1


def imex_euler(f: np.ndarray, tr: np.ndarray, dt: float, eps: float, plan: spectral.Plan,
               project: bool = True) -> np.ndarray:
    """One penalised first-order IMEX step of the Boltzmann layer (eq. 1002),
    Q(f^n) from the spectral oracle (projected on the invariants if asked)."""
    q = spectral.collide(f, plan)
    if project:
        q = spectral.project(q, plan.n, plan.L)
    return imex_combine(f, tr, q, dt, eps, plan.L)
