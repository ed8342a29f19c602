"""FP64 oracle of the fast spectral operator for Maxwell molecules in two
velocity dimensions (Sec. 4.4.1, the 2d case).

TEST INFRASTRUCTURE ONLY (see package doc).

What is computed, per spatial cell, for f sampled on v_j = (j - N/2) dv,
dv = 2L/N, j in [0,N)^2:

  1. fhat_k = N^-2 sum_j f_j exp(-i kappa_k . v_j), kappa_k = (pi/L) ktilde,
     ktilde in [-N/2, N/2)^2, the Nyquist lines (any ktilde_i = -N/2) set to
     zero, as in three dimensions.
  2. The Carleman kernel is constant in two dimensions for Maxwell molecules
     (the VHS exponent gamma = 0): Btilde = C, the paper taking C = 1.  In
     polar coordinates x = rho e, y = rho' e' with e . e' = 0 the spectral
     kernel becomes a half-circle integral
        Bhat_F(l, m) = int_0^pi phi(l . e_theta) phi(m . e_theta') d theta,
        e_theta = (cos theta, sin theta), e_theta' = e_{theta + pi/2},
        phi(s) = int_{-R}^{R} exp(i rho s) d rho = 2 R sinc(R s),
     and A equally spaced angles theta_p = pi p / A, p = 1..A, each of
     weight pi/A (spectrally accurate for this periodic integrand), give
        Bhat_F(l, m) = (pi/A) sum_p alpha_p(l) alpha'_p(m),
        alpha_p(l) = phi(l . e_theta_p), alpha'_p(m) = phi(m . e_theta_p').
  3. Gain: per angle, A_p = IDFT(alpha_p fhat) and A'_p = IDFT(alpha'_p fhat)
     are real (phi is even), Q+_j = (pi/A) sum_p A_p,j A'_p,j.
  4. Loss: Bhat_M(m) = Bhat_F(m, m), Lambda = IDFT(Bhat_M fhat), and the loss
     is fN Lambda, fN = IDFT(fhat) the truncated series.
  5. Q_j = C (Q+_j - fN_j Lambda_j).

The projection on the collision invariants of two velocity dimensions,
(1, v1, v2, |v|^2), restores what periodisation loses (Sec. 2.1).  Library
routines used: matrix products and a 4x4 linear solve.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

from . import spectral


@dataclass
class Plan2D:
    """Grid (n, L), truncation R, number of angles A, kernel constant C."""
    n: int
    L: float
    R: float
    A: int
    kernel_c: float = 1.0

    @property
    def weight(self) -> float:
        return math.pi / self.A

    def angles(self) -> np.ndarray:
        return math.pi * np.arange(1, self.A + 1) / self.A


def make_plan(n: int, L: float = 8.0, R: float | None = None, A: int = 32, kernel_c: float = 1.0) -> Plan2D:
    return Plan2D(n, L, spectral.default_R(L) if R is None else R, A, kernel_c)


def nyquist_mask(n: int) -> np.ndarray:
    nyq = np.arange(n) == n // 2
    return nyq[:, None] | nyq[None, :]


def forward(f: np.ndarray, n: int, L: float) -> np.ndarray:
    """fhat_k = n^-2 sum_j f_j exp(-i kappa_k . v_j), Nyquist lines zeroed."""
    E = np.exp(-1j * np.outer(spectral.wavenumbers(n, L), spectral.velocity_nodes(n, L)))
    g = E @ f.astype(np.complex128) @ E.T / float(n) ** 2
    g[nyquist_mask(n)] = 0.0
    return g


def inverse(g: np.ndarray, n: int, L: float) -> np.ndarray:
    """sum_k g_k exp(i kappa_k . v_j) on the grid."""
    E = np.exp(1j * np.outer(spectral.velocity_nodes(n, L), spectral.wavenumbers(n, L)))
    return E @ g @ E.T


def phi(s, R: float) -> np.ndarray:
    """phi(s) = int_{-R}^{R} exp(i rho s) d rho = 2 R sinc(R s)."""
    return 2.0 * R * np.sinc(R * np.asarray(s, dtype=np.float64) / math.pi)


def multipliers(plan: Plan2D, p: int):
    """(alpha_p, alpha'_p) on the [k1][k2] grid for the angle theta_p, p in
    0..A-1 standing for theta = pi (p + 1) / A."""
    th = plan.angles()[p]
    k = spectral.wavenumbers(plan.n, plan.L)
    K1, K2 = np.meshgrid(k, k, indexing="ij")
    a = phi(K1 * math.cos(th) + K2 * math.sin(th), plan.R)
    b = phi(-K1 * math.sin(th) + K2 * math.cos(th), plan.R)
    return a, b


def bhat_m(plan: Plan2D) -> np.ndarray:
    out = np.zeros((plan.n, plan.n))
    for p in range(plan.A):
        a, b = multipliers(plan, p)
        out += plan.weight * a * b
    return out


def collide_parts(f: np.ndarray, plan: Plan2D):
    """(Q, C Q+, C fN Lambda) of one cell."""
    n, L = plan.n, plan.L
    fh = forward(f, n, L)
    gain = np.zeros((n, n))
    for p in range(plan.A):
        a, b = multipliers(plan, p)
        ga = inverse(a * fh, n, L)
        gb = inverse(b * fh, n, L)
        gain += plan.weight * ga.real * gb.real
    lam = inverse(bhat_m(plan) * fh, n, L).real
    fN = inverse(fh, n, L).real
    c = plan.kernel_c
    return c * (gain - fN * lam), c * gain, c * fN * lam


def collide(f: np.ndarray, plan: Plan2D) -> np.ndarray:
    return collide_parts(f, plan)[0]


def moment_matrix(n: int, L: float) -> np.ndarray:
    """C (4 x n^2): rows 1, v1, v2, |v|^2 (the collision invariants in two
    velocity dimensions)."""
    v = spectral.velocity_nodes(n, L)
    V1, V2 = np.meshgrid(v, v, indexing="ij")
    return np.stack([np.ones(n * n), V1.ravel(), V2.ravel(), (V1 * V1 + V2 * V2).ravel()])


def project(q: np.ndarray, n: int, L: float) -> np.ndarray:
    """Q - C^T (C C^T)^-1 C Q: the least-squares correction onto {C Q = 0}."""
    C = moment_matrix(n, L)
    lam = np.linalg.solve(C @ C.T, C @ q.ravel())
    return (q.ravel() - C.T @ lam).reshape(q.shape)


def moment_drift(q: np.ndarray, n: int, L: float) -> float:
    C = moment_matrix(n, L)
    qq = q.ravel()
    return float(np.max(np.abs(C @ qq) / (np.abs(C) @ np.abs(qq))))


def collide_batch(f: np.ndarray, plan: Plan2D, project_out: bool = True) -> np.ndarray:
    out = np.empty(f.shape, dtype=np.float64)
    for c in range(f.shape[0]):
        q = collide(f[c], plan)
        out[c] = project(q, plan.n, plan.L) if project_out else q
    return out
