"""Seeded synthetic inputs shared by the oracle, the tests and the benchmark.

This module holds no arithmetic of the collision method: it only evaluates
Maxwellian-shaped distributions on the velocity grid and draws macroscopic
fields.  The velocity grid follows the discrete-velocity layout of Sec. 4.1
(v_j = (j - N/2) * dv on [-L, L)^3, index i3 fastest); the Maxwellian is the
equilibrium of hypothesis (H3) in Sec. 2.

Workload recipes (all seeded with numpy.random.default_rng):
  * ``bimaxwellian_cell``   single cell, mix of two Maxwellians
                            (densities U[0.5,1.5], means U[-1,1]^3,
                            temperatures U[0.5,2]).
  * ``shock_batch``         cells shaped like a Mach 2-2.9 Mott-Smith shock
                            profile plus an anisotropic bi-Maxwellian
                            perturbation (density ratio <= 3,
                            temperature ratio <= 3.5).
  * ``bow_shock_field``     2D macro field (rho, ux, uy, T) with a curved
                            shock in front of a round body, moving a quarter
                            cell per step; stands in for the obstacle flows of
                            Sec. 5 (Tests 2 and 4).
  * ``serving_requests``    request stream of several simulations with grid
                            sizes N in {16,24,32,48} and Poisson cell counts.
  * ``bimaxwellian2d_batch`` two-velocity-dimension cells (a Maxwellian plus an
                            anisotropic Gaussian) for the 2D Maxwell-molecule
                            operator.
"""
from __future__ import annotations

import math

import numpy as np

GAMMA_GAS = 5.0 / 3.0  # monatomic gas, Xi = 5/3 as in the Euler closure of Sec. 4.2


def velocity_axis(n: int, L: float) -> np.ndarray:
    """1D velocity nodes v_j = (j - n/2) * 2L/n, j = 0..n-1 (Sec. 4.1)."""
    dv = 2.0 * L / n
    return (np.arange(n, dtype=np.float64) - n // 2) * dv


def maxwellian(n: int, L: float, rho: float, u, T: float) -> np.ndarray:
    """M_{rho,u,T}(v) = rho/(2 pi T)^{3/2} exp(-|v-u|^2/(2T)) on the n^3 grid
    (hypothesis (H3), Sec. 2).  Returns float64 [n][n][n], index i3 fastest."""
    v = velocity_axis(n, L)
    u = np.asarray(u, dtype=np.float64)
    e1 = (v - u[0]) ** 2
    e2 = (v - u[1]) ** 2
    e3 = (v - u[2]) ** 2
    r2 = e1[:, None, None] + e2[None, :, None] + e3[None, None, :]
    return rho / (2.0 * math.pi * T) ** 1.5 * np.exp(-r2 / (2.0 * T))


def anisotropic_gaussian(n: int, L: float, rho: float, u, Tpar: float, Tperp: float,
                         axis) -> np.ndarray:
    """Gaussian with temperature Tpar along the unit vector ``axis`` and Tperp
    across it (a bi-Maxwellian-type perturbation)."""
    v = velocity_axis(n, L)
    a = np.asarray(axis, dtype=np.float64)
    a = a / np.linalg.norm(a)
    u = np.asarray(u, dtype=np.float64)
    V1, V2, V3 = np.meshgrid(v - u[0], v - u[1], v - u[2], indexing="ij")
    par = V1 * a[0] + V2 * a[1] + V3 * a[2]
    r2 = V1 * V1 + V2 * V2 + V3 * V3
    perp2 = r2 - par * par
    norm = rho / ((2.0 * math.pi) ** 1.5 * math.sqrt(Tpar) * Tperp)
    return norm * np.exp(-par * par / (2.0 * Tpar) - perp2 / (2.0 * Tperp))


def bimaxwellian_cell(n: int, L: float, rng: np.random.Generator) -> np.ndarray:
    """rho1 M(u1,T1) + rho2 M(u2,T2) with rho_i~U[0.5,1.5], u_i~U[-1,1]^3,
    T_i~U[0.5,2]."""
    f = np.zeros((n, n, n))
    for _ in range(2):
        rho = rng.uniform(0.5, 1.5)
        u = rng.uniform(-1.0, 1.0, size=3)
        T = rng.uniform(0.5, 2.0)
        f += maxwellian(n, L, rho, u, T)
    return f


def rankine_hugoniot(mach: float):
    """Density and temperature ratios across a normal shock, gas constant 5/3."""
    g = GAMMA_GAS
    m2 = mach * mach
    r_rho = (g + 1.0) * m2 / ((g - 1.0) * m2 + 2.0)
    r_p = (2.0 * g * m2 - (g - 1.0)) / (g + 1.0)
    return r_rho, r_p / r_rho


def shock_batch(ncells: int, n: int, L: float, seed: int) -> np.ndarray:
    """Cells across a Mott-Smith shock: f_c = (1-w_c) M_up + w_c M_down plus an
    anisotropic Gaussian perturbation.  Mach ~ U[2.0, 2.9] (density ratio
    <= 2.95, temperature ratio <= 3.48), upstream rho=1, T~U[0.5,0.6], shock
    normal seeded (x-aligned for even cells), frame shifted so the mixture
    velocity is near zero, position x_c = -3 + 6c/(ncells-1),
    w_c = (1 + tanh x_c)/2, perturbation amplitude <= 0.1 rho with
    Tpar/Tperp ~ U[0.8, 1.25]."""
    rng = np.random.default_rng(seed)
    out = np.empty((ncells, n, n, n))
    for c in range(ncells):
        mach = rng.uniform(2.0, 2.9)
        T1 = rng.uniform(0.5, 0.6)
        if c % 2 == 0:
            nrm = np.array([1.0, 0.0, 0.0])
        else:
            nrm = rng.normal(size=3)
            nrm /= np.linalg.norm(nrm)
        r_rho, r_T = rankine_hugoniot(mach)
        u1 = mach * math.sqrt(GAMMA_GAS * T1)
        rho2, T2, u2 = r_rho, r_T * T1, u1 / r_rho
        xc = -3.0 + 6.0 * c / max(ncells - 1, 1)
        w = 0.5 * (1.0 + math.tanh(xc))
        # shift frame so that the mixture's mean velocity is ~0
        ubar = ((1.0 - w) * u1 + w * rho2 * u2) / ((1.0 - w) + w * rho2)
        f = (1.0 - w) * maxwellian(n, L, 1.0, (u1 - ubar) * nrm, T1)
        f += w * maxwellian(n, L, rho2, (u2 - ubar) * nrm, T2)
        amp = rng.uniform(0.0, 0.1)
        ratio = rng.uniform(0.8, 1.25)
        Tm = (1.0 - w) * T1 + w * T2
        ax = rng.normal(size=3)
        f += amp * anisotropic_gaussian(n, L, 1.0, rng.uniform(-0.3, 0.3, 3),
                                        Tm * ratio, Tm, ax)
        out[c] = f
    return out


def bimaxwellian_batch(ncells: int, n: int, L: float, seed: int) -> np.ndarray:
    rng = np.random.default_rng(seed)
    return np.stack([bimaxwellian_cell(n, L, rng) for _ in range(ncells)])


def bkw_profile(n: int, L: float, K: float) -> np.ndarray:
    """The BKW similarity profile f_K(v) = (2 pi K)^{-3/2} exp(-|v|^2/(2K))
    [(5K-3)/(2K) + (1-K)|v|^2/(2K^2)], K >= 3/5 (a known exact solution of the
    space-homogeneous equation for Maxwell-type kernels)."""
    v = velocity_axis(n, L)
    r2 = v[:, None, None] ** 2 + v[None, :, None] ** 2 + v[None, None, :] ** 2
    return (2.0 * math.pi * K) ** -1.5 * np.exp(-r2 / (2.0 * K)) * (
        (5.0 * K - 3.0) / (2.0 * K) + (1.0 - K) * r2 / (2.0 * K * K))


def maxwellian2d(n: int, L: float, rho: float, u, T: float) -> np.ndarray:
    """Two-dimensional Maxwellian rho/(2 pi T) exp(-|v-u|^2/(2T)) on the n^2
    grid v_j = (j - n/2) * 2L/n.  Returns float64 [n][n], index i2 fastest."""
    v = velocity_axis(n, L)
    r2 = (v[:, None] - u[0]) ** 2 + (v[None, :] - u[1]) ** 2
    return rho / (2.0 * math.pi * T) * np.exp(-r2 / (2.0 * T))


def gaussian2d(n: int, L: float, rho: float, u, T1: float, T2: float, angle: float) -> np.ndarray:
    """Anisotropic 2D Gaussian: temperature T1 along the direction at ``angle``
    (radians from the v1 axis) and T2 across it."""
    v = velocity_axis(n, L)
    V1, V2 = np.meshgrid(v - u[0], v - u[1], indexing="ij")
    a = V1 * math.cos(angle) + V2 * math.sin(angle)
    b = -V1 * math.sin(angle) + V2 * math.cos(angle)
    return rho / (2.0 * math.pi * math.sqrt(T1 * T2)) * np.exp(-a * a / (2.0 * T1) - b * b / (2.0 * T2))


def bimaxwellian2d_batch(ncells: int, n: int, L: float, seed: int) -> np.ndarray:
    """Cells rho1 M(u1,T1) + rho2 G(u2,T2a,T2b) in two velocity dimensions:
    rho_i ~ U[0.5,1.5], u_i ~ U[-1,1]^2, T ~ U[0.5,2], the second component
    anisotropic (temperature ratio <= 3.5, random orientation)."""
    rng = np.random.default_rng(seed)
    out = np.empty((ncells, n, n))
    for c in range(ncells):
        rho1, rho2 = rng.uniform(0.5, 1.5, size=2)
        u1, u2 = rng.uniform(-1.0, 1.0, size=(2, 2))
        T1 = rng.uniform(0.5, 2.0)
        Ta = rng.uniform(0.5, 2.0)
        Tb = Ta * rng.uniform(1.0, 3.5)
        out[c] = maxwellian2d(n, L, rho1, u1, T1) + gaussian2d(n, L, rho2, u2, Ta, Tb, rng.uniform(0.0, math.pi))
    return out


def bow_shock_field(nx: int, ny: int, step: int, seed: int, noise: float = 0.01):
    """Macro fields (rho, ux, uy, T) on the unit square, [iy][ix] row-major.

    Free stream rho=1, T=0.5, Mach 2.5 along +x; a curved shock
    x_s(y) = 0.45 + 0.25*step/nx - 2.5 (y-0.5)^2 with tanh width 2 dx;
    post-shock state from the normal-shock relations; a round body at
    (0.6, 0.5), radius 0.08, with a thin stagnating layer around it; 1 %
    seeded low-mode noise whose phase advances with ``step``."""
    rng = np.random.default_rng(seed)
    dx = 1.0 / nx
    x = (np.arange(nx) + 0.5) * dx
    y = (np.arange(ny) + 0.5) / ny
    X, Y = np.meshgrid(x, y, indexing="xy")
    T1, rho1, mach = 0.5, 1.0, 2.5
    u1 = mach * math.sqrt(GAMMA_GAS * T1)
    r_rho, r_T = rankine_hugoniot(mach)
    xs = 0.45 + 0.25 * step * dx - 2.5 * (Y - 0.5) ** 2
    s = 0.5 * (1.0 + np.tanh((X - xs) / (2.0 * dx)))
    rho = rho1 * (1.0 + (r_rho - 1.0) * s)
    T = T1 * (1.0 + (r_T - 1.0) * s)
    # normal of the shock curve: (1, 5 (y-0.5)) / |.|
    nxv = 1.0 / np.sqrt(1.0 + (5.0 * (Y - 0.5)) ** 2)
    nyv = 5.0 * (Y - 0.5) * nxv
    un_post = u1 / r_rho
    ux = u1 * (1.0 - s) + s * (u1 - (u1 - un_post) * nxv * nxv)
    uy = s * (-(u1 - un_post) * nxv * nyv)
    rc = np.sqrt((X - 0.6) ** 2 + (Y - 0.5) ** 2)
    body = 0.08
    layer = np.exp(-np.maximum(rc - body, 0.0) / (3.0 * dx))
    ux = ux * (1.0 - layer)
    uy = uy * (1.0 - layer)
    T = T + 0.5 * layer * T
    phase = rng.uniform(0.0, 2.0 * math.pi, size=4) + 0.3 * step
    modes = (np.sin(2 * math.pi * X + phase[0]) * np.cos(2 * math.pi * Y + phase[1])
             + np.sin(4 * math.pi * X + phase[2]) * np.sin(2 * math.pi * Y + phase[3]))
    rho = rho * (1.0 + noise * 0.5 * modes)
    T = T * (1.0 + noise * 0.5 * np.roll(modes, 3, axis=1))
    return (np.ascontiguousarray(rho), np.ascontiguousarray(ux),
            np.ascontiguousarray(uy), np.ascontiguousarray(T))


def random_macro_field(nx: int, ny: int, seed: int, amp: float = 0.3):
    """Smooth random positive macro fields for mask parity tests."""
    rng = np.random.default_rng(seed)
    X, Y = np.meshgrid(np.arange(nx) / nx, np.arange(ny) / ny, indexing="xy")
    def smooth():
        a = rng.normal(size=(3, 3))
        f = np.zeros_like(X)
        for i in range(3):
            for j in range(3):
                f += a[i, j] * np.sin(2 * math.pi * (i + 1) * X + rng.uniform(0, 6)) * \
                    np.cos(2 * math.pi * (j + 1) * Y + rng.uniform(0, 6))
        return f / 9.0
    rho = 1.0 + amp * np.tanh(smooth()) + 0.02 * rng.normal(size=X.shape)
    T = 1.0 + amp * np.tanh(smooth()) + 0.02 * rng.normal(size=X.shape)
    ux = smooth() + 0.05 * rng.normal(size=X.shape)
    uy = smooth() + 0.05 * rng.normal(size=X.shape)
    return (np.ascontiguousarray(rho), np.ascontiguousarray(ux),
            np.ascontiguousarray(uy), np.ascontiguousarray(T))


def serving_requests(nclients: int, per_client: int, seed: int,
                     sizes=(16, 24, 32, 48), mean_cells: int = 512,
                     lo: int = 16, hi: int = 4096):
    """Request descriptors (client, N, ncells) with N uniform over ``sizes`` and
    cell counts ~ Poisson(mean) clipped to [lo, hi]."""
    rng = np.random.default_rng(seed)
    reqs = []
    for c in range(nclients):
        for _ in range(per_client):
            n = int(rng.choice(sizes))
            k = int(np.clip(rng.poisson(mean_cells), lo, hi))
            reqs.append((c, n, k))
    return reqs
