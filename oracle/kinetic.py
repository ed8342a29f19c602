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
  imex_euler   the penalised scheme of Sec. 4.4 (eq. (4.24)): with the transport
               term tr = v . grad_x f^n given,
                 g = f^n - dt tr,  U^{n+1} = int phi g (phi = 1, v, |v|^2),
                 beta = 2 pi rho^{n+1},  P(h) = beta (M[h] - h),
                 f^{n+1} = eps/(eps + beta dt) g
                           + dt (Q(f^n) - P(f^n)) / (eps + beta dt)
                           + beta dt/(eps + beta dt) M^{n+1},
               M^{n+1} the Maxwellian of U^{n+1}.
  pr222_step   the same penalised splitting integrated with the second-order
               PR(2,2,2) IMEX Runge-Kutta tableaux (Sec. 4.3), transport given
               as a function of the stage value.
  esbgk_*      the ES-BGK operator Q_ES = nu (G[f] - f) with the corrected
               Gaussian G of Sec. 2.2, and its first-order IMEX step solved
               explicitly (Sec. 4.3).
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
    """The update of eq. (4.24) given Q(f^n) (any array q) and the transport term."""
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
    """One penalised first-order IMEX step of the Boltzmann layer (eq. (4.24)),
    Q(f^n) from the spectral oracle (projected on the invariants if asked)."""
    q = spectral.collide(f, plan)
    if project:
        q = spectral.project(q, plan.n, plan.L)
    return imex_combine(f, tr, q, dt, eps, plan.L)


# ---------------------------------------------------------------- ES-BGK (Sec. 2.2)
def second_moments(h: np.ndarray, n: int, L: float) -> np.ndarray:
    """S = int v (x) v h, a symmetric 3x3 matrix."""
    V = _grid(n, L)
    w = V[3]
    return np.array([[w * (V[a] * V[b] * h).sum() for b in range(3)] for a in range(3)])


def stress(f: np.ndarray, n: int, L: float):
    """(rho, u, Theta) with rho Theta = int (v - u) (x) (v - u) f (Sec. 2.2)."""
    rho, u, _ = moments(f, n, L)
    V = _grid(n, L)
    w = V[3]
    th = np.array([[w * ((V[a] - u[a]) * (V[b] - u[b]) * f).sum() for b in range(3)] for a in range(3)]) / rho
    return rho, u, th


def anisotropic_gaussian(rho: float, u, tau: np.ndarray, n: int, L: float) -> np.ndarray:
    """G = rho / sqrt(det(2 pi Tau)) exp(-(v - u) Tau^-1 (v - u) / 2)."""
    V1, V2, V3, _ = _grid(n, L)
    d = np.stack([V1 - u[0], V2 - u[1], V3 - u[2]], axis=-1)
    ti = np.linalg.inv(tau)
    quad = np.einsum("...a,ab,...b->...", d, ti, d)
    return rho / math.sqrt(np.linalg.det(2.0 * math.pi * tau)) * np.exp(-0.5 * quad)


def esbgk_frequency(rho: float, T: float, beta: float, mu0: float) -> float:
    """nu(rho, T): relaxation rate whose ES-BGK viscosity rho T / (nu (1 - beta))
    is the hard-sphere mu = mu0 sqrt(T)."""
    return rho * math.sqrt(T) / (mu0 * (1.0 - beta))


def esbgk_tensor(T: float, theta: np.ndarray, beta: float) -> np.ndarray:
    """Tau = (1 - beta) T I + beta Theta (Sec. 2.2)."""
    return (1.0 - beta) * T * np.eye(3) + beta * theta


def esbgk_gaussian(f: np.ndarray, n: int, L: float, beta: float) -> np.ndarray:
    """G[f] of Sec. 2.2 from f's own density, velocity and stress."""
    rho, u, th = stress(f, n, L)
    T = np.trace(th) / 3.0
    return anisotropic_gaussian(rho, u, esbgk_tensor(T, th, beta), n, L)


def esbgk_collide(f: np.ndarray, n: int, L: float, beta: float, mu0: float) -> np.ndarray:
    """Q_ES(f) = nu(rho, T) (G[f] - f) (Sec. 2.2)."""
    rho, u, th = stress(f, n, L)
    T = np.trace(th) / 3.0
    G = anisotropic_gaussian(rho, u, esbgk_tensor(T, th, beta), n, L)
    return esbgk_frequency(rho, T, beta, mu0) * (G - f)


def esbgk_imex_euler(f: np.ndarray, tr: np.ndarray, dt: float, eps: float, L: float, beta: float,
                     mu0: float) -> np.ndarray:
    """One first-order IMEX step of the ES-BGK layer (Sec. 4.3, after Filbet
    and Jin), solved explicitly:
      g = f^n - dt tr;  U^{n+1} = int phi g -> rho, u, T at n+1;  nu = nu(rho, T);
      Sigma^{n+1} = eps/(eps + (1-beta) nu dt) int v (x) v g
                    + (1-beta) nu dt/(eps + (1-beta) nu dt) rho (T I + u (x) u);
      Theta^{n+1} = Sigma^{n+1}/rho - u (x) u;  Tau = (1-beta) T I + beta Theta;
      f^{n+1} = eps/(eps + nu dt) g + nu dt/(eps + nu dt) G(rho, u, Tau)."""
    n = f.shape[0]
    g = f - dt * tr
    U = conserved(g, n, L)
    rho = U[0]
    u = U[1:4] / rho
    T = (U[4] / rho - u @ u) / 3.0
    nu = esbgk_frequency(rho, T, beta, mu0)
    a = eps / (eps + (1.0 - beta) * nu * dt)
    sigma = a * second_moments(g, n, L) + (1.0 - a) * rho * (T * np.eye(3) + np.outer(u, u))
    theta = sigma / rho - np.outer(u, u)
    G = anisotropic_gaussian(rho, u, esbgk_tensor(T, theta, beta), n, L)
    c = eps / (eps + nu * dt)
    return c * g + (1.0 - c) * G


# ---------------------------------------------------------------- PR(2,2,2) (Sec. 4.3-4.4)
PR_C = 1.0 / math.sqrt(2.0)
PR_DELTA = 1.0 - 1.0 / (2.0 * PR_C)
# explicit tableau (c~, A~, w~) and implicit tableau (c, A, w) of PR(2,2,2)
PR_A_EXP = np.array([[0.0, 0.0], [1.0, 0.0]])
PR_W_EXP = np.array([0.5, 0.5])
PR_A_IMP = np.array([[1.0 - PR_C, 0.0], [PR_C - PR_DELTA, PR_DELTA]])
PR_W_IMP = np.array([0.5, 0.5])


def penalty_solve(r: np.ndarray, h: float, eps: float, L: float) -> np.ndarray:
    """Solution Y of Y = r + (h / eps) P(Y), P(Y) = beta (M[Y] - Y), beta = 2 pi rho:
    P conserves (1, v, |v|^2), so M[Y] = M[r] and rho(Y) = rho(r), and
    Y = (eps r + h beta M[r]) / (eps + h beta)."""
    n = r.shape[0]
    M, rho = maxwellian_of_conserved(conserved(r, n, L), n, L)
    beta = 2.0 * math.pi * rho
    return (eps * r + h * beta * M) / (eps + h * beta)


def penalty(y: np.ndarray, L: float) -> np.ndarray:
    """P(y) = beta (M[y] - y), beta = 2 pi rho(y) (the implicit part of the penalised scheme)."""
    n = y.shape[0]
    M, rho = maxwellian_of_conserved(conserved(y, n, L), n, L)
    return 2.0 * math.pi * rho * (M - y)


def pr222_step(y: np.ndarray, transport, dt: float, eps: float, plan: spectral.Plan,
               project: bool = True) -> np.ndarray:
    """One PR(2,2,2) step of y' = q(y) + g(y)/eps with the explicit part
    q(y) = -transport(y) + (Q(y) - P(y))/eps and the implicit part g = P,
    following the IMEX Runge-Kutta form of Sec. 4.3 with the tableaux printed
    there (C = 1/sqrt 2); each implicit stage is solved by penalty_solve."""
    L = plan.L

    def Q(z):
        q = spectral.collide(z, plan)
        return spectral.project(q, plan.n, L) if project else q

    def q_exp(z):
        return -transport(z) + (Q(z) - penalty(z, L)) / eps

    Y, qs, gs = [], [], []
    for i in range(2):
        r = y.copy()
        for j in range(i):
            r = r + dt * PR_A_EXP[i, j] * qs[j] + dt * PR_A_IMP[i, j] * gs[j] / eps
        Yi = penalty_solve(r, dt * PR_A_IMP[i, i], eps, L)
        Y.append(Yi)
        qs.append(q_exp(Yi))
        gs.append(penalty(Yi, L))
    out = y.copy()
    for i in range(2):
        out = out + dt * PR_W_EXP[i] * qs[i] + dt * PR_W_IMP[i] * gs[i] / eps
    return out


def esbgk_stage_solve(r: np.ndarray, h: float, eps: float, L: float, beta: float, mu0: float) -> np.ndarray:
    """Solution Y of Y = r + (h/eps) Q_ES(Y): the first-order ES-BGK step with
    the transport removed (Q_ES conserves (1, v, |v|^2), so rho, u, T and nu of Y
    are those of r, and the stress follows from the second-moment equation)."""
    return esbgk_imex_euler(r, np.zeros_like(r), h, eps, L, beta, mu0)


def esbgk_pr222_step(y: np.ndarray, transport, dt: float, eps: float, L: float, beta: float,
                     mu0: float) -> np.ndarray:
    """One PR(2,2,2) step of y' = -transport(y) + Q_ES(y)/eps (explicit part:
    transport; implicit part: the ES-BGK relaxation), with the tableaux of
    Sec. 4.3; each implicit stage solved by esbgk_stage_solve."""
    n = y.shape[0]
    Y, qs, gs = [], [], []
    for i in range(2):
        r = y.copy()
        for j in range(i):
            r = r + dt * PR_A_EXP[i, j] * qs[j] + dt * PR_A_IMP[i, j] * gs[j] / eps
        Yi = esbgk_stage_solve(r, dt * PR_A_IMP[i, i], eps, L, beta, mu0)
        Y.append(Yi)
        qs.append(-transport(Yi))
        gs.append(esbgk_collide(Yi, n, L, beta, mu0))
    out = y.copy()
    for i in range(2):
        out = out + dt * PR_W_EXP[i] * qs[i] + dt * PR_W_IMP[i] * gs[i] / eps
    return out


def realizability_matrix(f: np.ndarray, n: int, L: float) -> np.ndarray:
    """Moment realizability matrix of the appendix (Moment realizability
    matrix): with V = (v - u)/sqrt(T) and the reduced invariants
    m = (1, V, (2/5)^(1/2) (|V|^2/2 - 5/2)),  M = (1/rho) int m (x) m f dv
    (5 x 5; u and T from moments(f))."""
    rho, u, T = moments(f, n, L)
    v1, v2, v3, dv3 = _grid(n, L)
    s = 1.0 / math.sqrt(T)
    V = [(v1 - u[0]) * s, (v2 - u[1]) * s, (v3 - u[2]) * s]
    m = [np.ones_like(v1)] + V + [math.sqrt(2.0 / 5.0) * ((V[0] ** 2 + V[1] ** 2 + V[2] ** 2) / 2.0 - 2.5)]
    M = np.empty((5, 5))
    for i in range(5):
        for j in range(5):
            M[i, j] = (m[i] * m[j] * f).sum() * dv3 / rho
    return M


def reduced_realizability(M: np.ndarray):
    """Split M into Abar (M[1:4,1:4] - I), Bbar (M[1:4,4] / (2/5)^(1/2)) and
    Cbar (M[4,4]), and return (Cbar, V) with the Schur-complement form
    V = I + Abar - (2/(5 Cbar)) / (1 - 2/(5 Cbar)) Bbar (x) Bbar
    (valid for Cbar > 2/5; Cbar = 1 gives I + Abar - (2/3) Bbar (x) Bbar)."""
    A = M[1:4, 1:4] - np.eye(3)
    B = M[1:4, 4] / math.sqrt(2.0 / 5.0)
    C = M[4, 4]
    k = 2.0 / (5.0 * C)
    return C, np.eye(3) + A - (k / (1.0 - k)) * np.outer(B, B)
