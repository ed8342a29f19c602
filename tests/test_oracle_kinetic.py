"""Pins of the kinetic oracle (macroscopic fields, Maxwellian, L1 distance,
penalised IMEX update) against closed forms and exact identities."""
import math

import numpy as np
import pytest

import bz_inputs as gen
from oracle import directions, kinetic, spectral


def grid(n, L):
    return kinetic._grid(n, L)


def test_moments_of_a_maxwellian():
    # trapezoidal sums of a resolved Gaussian are exact to rounding
    n, L = 48, 10.0
    f = kinetic.maxwellian(1.7, [0.4, -0.3, 0.25], 0.8, n, L)
    rho, u, T = kinetic.moments(f, n, L)
    assert abs(rho - 1.7) <= 1e-13 * 1.7
    assert np.abs(u - [0.4, -0.3, 0.25]).max() <= 1e-13
    assert abs(T - 0.8) <= 1e-12


def test_moments_of_a_mixture():
    # rho = sum rho_i, rho u = sum rho_i u_i, 3 rho T + rho |u|^2 = sum rho_i (3 T_i + |u_i|^2)
    n, L = 48, 10.0
    parts = [(0.9, np.array([1.2, 0.0, -0.5]), 0.6), (0.6, np.array([-0.8, 0.7, 0.3]), 1.4)]
    f = sum(kinetic.maxwellian(r, u, T, n, L) for r, u, T in parts)
    rho_x = sum(r for r, _, _ in parts)
    u_x = sum(r * u for r, u, _ in parts) / rho_x
    T_x = (sum(r * (3 * T + u @ u) for r, u, T in parts) - rho_x * u_x @ u_x) / (3 * rho_x)
    rho, u, T = kinetic.moments(f, n, L)
    assert abs(rho - rho_x) <= 1e-13
    assert np.abs(u - u_x).max() <= 1e-13
    assert abs(T - T_x) <= 1e-12


def test_l1_of_a_maxwellian_vanishes():
    n, L = 48, 10.0
    f = kinetic.maxwellian(1.1, [0.3, 0.1, -0.2], 1.2, n, L)
    assert kinetic.l1_distance(f, n, L) <= 1e-12


@pytest.mark.parametrize("kind", ["normal_stress", "shear_stress"])
def test_l1_closed_form(kind):
    # f = M (1 + a h) with h orthogonal to 1, v, |v|^2 under M keeps M[f] = M, so
    # ||f - M||_1 = rho |a| E|h|:  E|X^2 - Y^2| = 4T/pi,  E|XY| = 2T/pi  (X, Y ~ N(0, T))
    n, L, rho, u, T, a = 64, 8.0, 1.3, np.array([0.2, -0.1, 0.3]), 1.0, 0.1
    V1, V2, V3, _ = grid(n, L)
    M = kinetic.maxwellian(rho, u, T, n, L)
    if kind == "normal_stress":
        h, mean_abs = ((V1 - u[0]) ** 2 - (V2 - u[1]) ** 2) / T, 4.0 / math.pi
    else:
        h, mean_abs = (V1 - u[0]) * (V2 - u[1]) / T, 2.0 / math.pi
    f = M * (1.0 + a * h)
    r2, u2, T2 = kinetic.moments(f, n, L)
    assert abs(r2 - rho) <= 1e-12 and np.abs(u2 - u).max() <= 1e-12 and abs(T2 - T) <= 1e-10
    # the integrand has kinks on the planes where h changes sign: O(dv^2) quadrature error
    assert abs(kinetic.l1_distance(f, n, L) / (rho * a * mean_abs) - 1.0) <= 5e-3


def test_conserved_and_maxwellian_of_conserved():
    n, L = 48, 10.0
    f = kinetic.maxwellian(0.7, [0.5, -0.2, 0.1], 0.9, n, L)
    U = kinetic.conserved(f, n, L)
    assert np.allclose(U, [0.7, 0.35, -0.14, 0.07, 0.7 * (3 * 0.9 + 0.25 + 0.04 + 0.01)], rtol=0, atol=1e-13)
    M, rho = kinetic.maxwellian_of_conserved(U, n, L)
    assert abs(rho - 0.7) <= 1e-14
    assert np.abs(M - f).max() <= 1e-13 * f.max()


def random_transport(n, L, seed):
    # a smooth, seeded stand-in for v . grad_x f (any array works for the identities below)
    rng = np.random.default_rng(seed)
    V1, V2, V3, _ = grid(n, L)
    c = rng.uniform(-1, 1, 3)
    return (c[0] * V1 + c[1] * V2 + c[2] * V3) * kinetic.maxwellian(1.0, rng.uniform(-0.5, 0.5, 3), 1.0, n, L)


def test_imex_homogeneous_closed_form():
    # tr = 0: U^{n+1} = U^n, M^{n+1} = M^n, so f^{n+1} = f + dt Q / (eps + 2 pi rho dt)
    n, L = 32, 8.0
    f = gen.shock_batch(1, n, L, seed=11)[0]
    q = np.random.default_rng(3).standard_normal(f.shape) * 1e-3
    dt, eps = 0.01, 0.05
    rho = kinetic.moments(f, n, L)[0]
    out = kinetic.imex_combine(f, np.zeros_like(f), q, dt, eps, L)
    want = f + dt * q / (eps + 2 * math.pi * rho * dt)
    assert np.abs(out - want).max() <= 1e-13 * np.abs(f).max()


def test_imex_limits():
    n, L = 48, 10.0
    f = kinetic.maxwellian(1.0, [0.2, 0.0, -0.1], 1.0, n, L)
    tr = random_transport(n, L, 5)
    dt = 0.02
    g = f - dt * tr
    # eps >> beta dt: free transport
    out = kinetic.imex_combine(f, tr, np.zeros_like(f), dt, 1e12, L)
    assert np.abs(out - g).max() <= 1e-10 * np.abs(g).max()
    # eps -> 0 from equilibrium: the Maxwellian of U^{n+1} (asymptotic preservation)
    out = kinetic.imex_combine(f, tr, np.zeros_like(f), dt, 1e-14, L)
    M1, _ = kinetic.maxwellian_of_conserved(kinetic.conserved(g, n, L), n, L)
    assert np.abs(out - M1).max() <= 1e-11 * M1.max()


def test_imex_conserves_the_transported_moments():
    # with Q free of the invariants: int phi f^{n+1} = U^{n+1} = int phi (f - dt tr)
    n, L = 48, 10.0
    f = kinetic.maxwellian(0.8, [0.3, -0.2, 0.0], 0.7, n, L) + kinetic.maxwellian(0.4, [-0.6, 0.4, 0.2], 1.3, n, L)
    tr = random_transport(n, L, 6)
    q = spectral.project(np.random.default_rng(7).standard_normal(f.shape) * 1e-2, n, L)
    dt, eps = 0.01, 0.02
    out = kinetic.imex_combine(f, tr, q, dt, eps, L)
    U1 = kinetic.conserved(f - dt * tr, n, L)
    assert np.abs(kinetic.conserved(out, n, L) - U1).max() <= 1e-12 * np.abs(U1).max()


def test_imex_euler_uses_the_projected_operator():
    n, L = 16, 8.0
    d, w = directions.icosa6()
    plan = spectral.Plan(n, L, spectral.default_R(L), 1.0, 4.0, d, w)
    f = gen.bimaxwellian_batch(1, n, L, seed=1)[0]
    dt, eps = 0.005, 0.1
    out = kinetic.imex_euler(f, np.zeros_like(f), dt, eps, plan)
    q = spectral.project(spectral.collide(f, plan), n, L)
    rho = kinetic.moments(f, n, L)[0]
    assert np.abs(out - (f + dt * q / (eps + 2 * math.pi * rho * dt))).max() <= 1e-13 * np.abs(f).max()


def test_imex_penalty_uses_the_new_density():
    # from equilibrium with q = 0: f^{n+1} = (eps g + beta dt M^{n+1}) / (eps + beta dt),
    # beta = 2 pi rho^{n+1} with rho^{n+1} the density of g = f - dt tr (transport changes it)
    n, L = 48, 10.0
    f = kinetic.maxwellian(1.0, [0.1, 0.2, 0.0], 0.9, n, L)
    V1, V2, V3, _ = grid(n, L)
    tr = 3.0 * f * (1.0 + 0.2 * V1)  # carries mass: rho(g) = (1 - 3 dt) rho(f) - ...
    dt, eps = 0.02, 0.03
    g = f - dt * tr
    M1, rho1 = kinetic.maxwellian_of_conserved(kinetic.conserved(g, n, L), n, L)
    assert abs(rho1 - 1.0) > 0.05
    beta = 2 * math.pi * rho1
    want = (eps * g + beta * dt * M1) / (eps + beta * dt)
    out = kinetic.imex_combine(f, tr, np.zeros_like(f), dt, eps, L)
    assert np.abs(out - want).max() <= 1e-12 * np.abs(want).max()


# ---------------------------------------------------------------- ES-BGK
def aniso(n, L, rho, u, cov):
    return kinetic.anisotropic_gaussian(rho, np.asarray(u), np.asarray(cov), n, L)


COV = np.array([[1.1, 0.2, -0.1], [0.2, 0.7, 0.05], [-0.1, 0.05, 0.9]])


def test_anisotropic_gaussian_moments():
    # density, velocity and stress of the sampled Gaussian are its parameters
    n, L = 48, 10.0
    f = aniso(n, L, 1.2, [0.3, -0.2, 0.1], COV)
    rho, u, th = kinetic.stress(f, n, L)
    assert abs(rho - 1.2) <= 1e-12
    assert np.abs(u - [0.3, -0.2, 0.1]).max() <= 1e-12
    assert np.abs(th - COV).max() <= 1e-11


def test_esbgk_limits_of_beta():
    n, L = 48, 10.0
    f = aniso(n, L, 1.2, [0.3, -0.2, 0.1], COV)
    # beta = 1: Tau = Theta, so G[f] = f and Q_ES = 0
    assert np.abs(kinetic.esbgk_gaussian(f, n, L, 1.0) - f).max() <= 1e-11 * f.max()
    # beta = 0: BGK, G[f] is the Maxwellian of f
    rho, u, T = kinetic.moments(f, n, L)
    assert abs(T - np.trace(COV) / 3) <= 1e-12
    M = kinetic.maxwellian(rho, u, T, n, L)
    assert np.abs(kinetic.esbgk_gaussian(f, n, L, 0.0) - M).max() <= 1e-12 * M.max()


def test_esbgk_conserves_and_relaxes_stress():
    # int (1, v, |v|^2) Q_ES = 0; the stress of G is (1 - beta) T I + beta Theta
    n, L, beta = 48, 10.0, -0.5
    f = gen.bimaxwellian_batch(1, n, L, seed=4)[0]
    f = f + aniso(n, L, 0.3, [0.5, 0.0, -0.4], COV)
    q = kinetic.esbgk_collide(f, n, L, beta, 1.0)
    U = kinetic.conserved(f, n, L)
    # exact up to the Gaussian tails cut at |v_i| = L (exp(-(L - 1)^2 / 4) ~ 1e-9 here)
    assert np.abs(kinetic.conserved(q, n, L)).max() <= 1e-8 * np.abs(U).max()
    rho, u, th = kinetic.stress(f, n, L)
    T = np.trace(th) / 3
    G = kinetic.esbgk_gaussian(f, n, L, beta)
    _, _, thG = kinetic.stress(G, n, L)
    assert np.abs(thG - ((1 - beta) * T * np.eye(3) + beta * th)).max() <= 1e-10
    # nu from the viscosity relation: rho T / (nu (1 - beta)) = mu0 sqrt(T)
    nu = kinetic.esbgk_frequency(rho, T, beta, 0.8)
    assert abs(rho * T / (nu * (1 - beta)) - 0.8 * math.sqrt(T)) <= 1e-14


def test_esbgk_imex_second_moments_are_consistent():
    # the explicit solution of the implicit step: int v (x) v f^{n+1} = Sigma^{n+1}
    # and int phi f^{n+1} = U^{n+1}
    n, L, beta, mu0 = 48, 10.0, -0.5, 1.0
    f = aniso(n, L, 1.0, [0.2, 0.1, -0.3], COV)
    tr = random_transport(n, L, 8)
    dt, eps = 0.02, 0.05
    out = kinetic.esbgk_imex_euler(f, tr, dt, eps, L, beta, mu0)
    g = f - dt * tr
    U = kinetic.conserved(g, n, L)
    assert np.abs(kinetic.conserved(out, n, L) - U).max() <= 1e-11 * np.abs(U).max()
    rho = U[0]
    u = U[1:4] / rho
    T = (U[4] / rho - u @ u) / 3
    nu = kinetic.esbgk_frequency(rho, T, beta, mu0)
    S_out = kinetic.second_moments(out, n, L)
    # Sigma solves Sigma = c S(g) + (1 - c) rho (Tau + u u) with Tau from Sigma (implicit)
    c = eps / (eps + nu * dt)
    tau = (1 - beta) * T * np.eye(3) + beta * (S_out / rho - np.outer(u, u))
    assert np.abs(S_out - (c * kinetic.second_moments(g, n, L) + (1 - c) * rho * (tau + np.outer(u, u)))).max() \
        <= 1e-10 * np.abs(S_out).max()


def test_esbgk_imex_limits():
    n, L, beta = 48, 10.0, -0.5
    f = aniso(n, L, 1.0, [0.2, 0.1, -0.3], COV)
    tr = random_transport(n, L, 9)
    dt = 0.02
    g = f - dt * tr
    assert np.abs(kinetic.esbgk_imex_euler(f, tr, dt, 1e12, L, beta, 1.0) - g).max() <= 1e-10 * np.abs(g).max()
    # eps -> 0: the stress relaxes to T I and f^{n+1} to the Maxwellian of U^{n+1}
    M1, _ = kinetic.maxwellian_of_conserved(kinetic.conserved(g, n, L), n, L)
    assert np.abs(kinetic.esbgk_imex_euler(f, tr, dt, 1e-14, L, beta, 1.0) - M1).max() <= 1e-10 * M1.max()


# ---------------------------------------------------------------- PR(2,2,2)
def test_pr222_tableaux_order_conditions():
    # both tableaux are second order and the pair satisfies the coupling conditions
    Ae, we, Ai, wi = kinetic.PR_A_EXP, kinetic.PR_W_EXP, kinetic.PR_A_IMP, kinetic.PR_W_IMP
    ce, ci = Ae.sum(axis=1), Ai.sum(axis=1)
    assert np.allclose(ci, [1 - kinetic.PR_C, kinetic.PR_C]) and np.allclose(ce, [0.0, 1.0])
    for w, c in ((we, ce), (wi, ci)):
        assert abs(w.sum() - 1.0) <= 1e-15 and abs(w @ c - 0.5) <= 1e-15
    assert abs(we @ ci - 0.5) <= 1e-15 and abs(wi @ ce - 0.5) <= 1e-15
    assert abs(kinetic.PR_DELTA - (1 - 1 / math.sqrt(2))) <= 1e-15  # the implicit diagonal gamma


def velocity_transport(n, L, c):
    # a transport stand-in that keeps the step local to the cell: T(y) = (c . v) y
    V1, V2, V3, _ = grid(n, L)
    w = c[0] * V1 + c[1] * V2 + c[2] * V3
    return lambda y: w * y


def test_pr222_conserves_the_transported_moments():
    n, L = 24, 8.0
    d, w = directions.icosa6()
    plan = spectral.Plan(n, L, spectral.default_R(L), 1.0, 4.0, d, w)
    f = kinetic.maxwellian(0.9, [0.2, -0.1, 0.0], 0.9, n, L) + kinetic.maxwellian(0.3, [-0.3, 0.2, 0.1], 1.1, n, L)
    T = velocity_transport(n, L, [0.3, -0.2, 0.1])
    dt, eps = 0.05, 0.1
    out = kinetic.pr222_step(f, T, dt, eps, plan)
    # rebuild the two stage values to know what the transport removed
    g = kinetic.PR_DELTA
    Y1 = kinetic.penalty_solve(f, g * dt, eps, L)
    q1 = spectral.project(spectral.collide(Y1, plan), n, L)
    R2 = f + dt * (-T(Y1) + (q1 - kinetic.penalty(Y1, L)) / eps) + dt * kinetic.PR_A_IMP[1, 0] * kinetic.penalty(Y1, L) / eps
    Y2 = kinetic.penalty_solve(R2, g * dt, eps, L)
    U = kinetic.conserved(f, n, L) - 0.5 * dt * (kinetic.conserved(T(Y1), n, L) + kinetic.conserved(T(Y2), n, L))
    assert np.abs(kinetic.conserved(out, n, L) - U).max() <= 1e-11 * np.abs(U).max()


def test_pr222_is_second_order_in_time():
    # homogeneous relaxation y' = Q(y)/eps: error against a fine RK4 solution drops ~4x per halving of dt
    n, L = 16, 8.0
    d, w = directions.icosa6()
    plan = spectral.Plan(n, L, spectral.default_R(L), 1.0, 4.0, d, w)
    f = gen.bimaxwellian_batch(1, n, L, seed=2)[0]
    eps, t_end = 5.0, 0.2  # beta dt / eps <= 0.13: the asymptotic (non-stiff) regime
    zero = lambda y: np.zeros_like(y)

    def Q(y):
        return spectral.project(spectral.collide(y, plan), n, L) / eps

    ref = f.copy()
    h = t_end / 64
    for _ in range(64):
        k1 = Q(ref); k2 = Q(ref + 0.5 * h * k1); k3 = Q(ref + 0.5 * h * k2); k4 = Q(ref + h * k3)
        ref = ref + h / 6 * (k1 + 2 * k2 + 2 * k3 + k4)
    errs = []
    for steps in (4, 8, 16):
        y = f.copy()
        for _ in range(steps):
            y = kinetic.pr222_step(y, zero, t_end / steps, eps, plan)
        errs.append(np.linalg.norm(y - ref))
    r1, r2 = errs[0] / errs[1], errs[1] / errs[2]
    assert 3.5 <= r1 <= 5.0 and 3.5 <= r2 <= 5.0, errs


def test_esbgk_stage_solve_solves_the_implicit_equation():
    # Y = r + (h/eps) Q_ES(Y), checked by evaluating Q_ES at the returned Y
    n, L, beta, mu0 = 48, 10.0, -0.5, 1.0
    r = aniso(n, L, 1.0, [0.2, 0.1, -0.3], COV)
    h, eps = 0.03, 0.05
    Y = kinetic.esbgk_stage_solve(r, h, eps, L, beta, mu0)
    res = Y - r - (h / eps) * kinetic.esbgk_collide(Y, n, L, beta, mu0)
    assert np.abs(res).max() <= 1e-10 * np.abs(Y).max()


def test_esbgk_pr222_order_and_conservation():
    n, L, beta, mu0 = 24, 8.0, -0.5, 1.0
    f = aniso(n, L, 1.0, [0.2, 0.1, -0.3], COV * 0.8) + aniso(n, L, 0.4, [-0.4, 0.2, 0.1], np.eye(3) * 0.9)
    T = velocity_transport(n, L, [0.3, -0.2, 0.1])
    eps, t_end = 2.0, 0.2
    # conservation: int phi y^{n+1} = int phi y - dt/2 int phi (T(Y1) + T(Y2)); checked through a step with T = 0
    zero = lambda y: np.zeros_like(y)
    out = kinetic.esbgk_pr222_step(f, zero, 0.05, eps, L, beta, mu0)
    U = kinetic.conserved(f, n, L)
    assert np.abs(kinetic.conserved(out, n, L) - U).max() <= 1e-10 * np.abs(U).max()
    # second order in time against RK4 on the same equation
    def rhs(y):
        return -T(y) + kinetic.esbgk_collide(y, n, L, beta, mu0) / eps
    ref = f.copy()
    h = t_end / 64
    for _ in range(64):
        k1 = rhs(ref); k2 = rhs(ref + 0.5 * h * k1); k3 = rhs(ref + 0.5 * h * k2); k4 = rhs(ref + h * k3)
        ref = ref + h / 6 * (k1 + 2 * k2 + 2 * k3 + k4)
    errs = []
    for steps in (4, 8, 16):
        y = f.copy()
        for _ in range(steps):
            y = kinetic.esbgk_pr222_step(y, T, t_end / steps, eps, L, beta, mu0)
        errs.append(np.linalg.norm(y - ref))
    r1, r2 = errs[0] / errs[1], errs[1] / errs[2]
    assert 3.5 <= r1 <= 5.0 and 3.5 <= r2 <= 5.0, errs


# ---------------------------------------------------------------- P13 (diagnostic)
def _thirteen_moment(n, L, rho, u, T, q, tau):
    """f = M (1 + phi) with the heat-flux and stress perturbation printed in
    the appendix (Moment realizability matrix)."""
    M = kinetic.maxwellian(rho, u, T, n, L)
    v = spectral.velocity_nodes(n, L)
    V = np.meshgrid(v, v, v, indexing="ij")
    c = [V[i] - u[i] for i in range(3)]
    c2 = c[0] ** 2 + c[1] ** 2 + c[2] ** 2
    cq = c[0] * q[0] + c[1] * q[1] + c[2] * q[2]
    ctc = sum(c[i] * tau[i, j] * c[j] for i in range(3) for j in range(3))
    phi = cq / (rho * T * T) * (c2 / (5 * T) - 1) + ctc / (2 * rho * T * T)
    return M * (1 + phi)


def test_p13_maxwellian_matrix_and_thirteen_moment_cbar():
    """At equilibrium M has the printed block form with Abar = Bbar = 0 and
    Cbar = 1; for f = M(1 + phi) (heat flux q, traceless stress tau) Cbar stays
    1 and the reduced matrix is I + Abar - (2/3) Bbar Bbar^T."""
    n, L = 32, 8.0
    f = kinetic.maxwellian(1.3, [0.2, -0.1, 0.3], 1.1, n, L)
    Mx = kinetic.realizability_matrix(f, n, L)
    ref = np.eye(5)
    ref[0, 4] = ref[4, 0] = -math.sqrt(2 / 5)
    assert np.abs(Mx - ref).max() <= 1e-9  # grid quadrature of fourth moments
    tau = np.array([[0.05, 0.02, 0.0], [0.02, -0.03, 0.01], [0.0, 0.01, -0.02]])
    f = _thirteen_moment(n, L, 1.0, np.zeros(3), 1.0, np.array([0.04, -0.02, 0.03]), tau)
    Mx = kinetic.realizability_matrix(f, n, L)
    C, V = kinetic.reduced_realizability(Mx)
    assert abs(C - 1.0) <= 5e-3  # Cbar = 1 to first order in (q, tau)
    A = Mx[1:4, 1:4] - np.eye(3)
    B = Mx[1:4, 4] / math.sqrt(2 / 5)
    V1 = np.eye(3) + A - (2 / 3) * np.outer(B, B)
    assert np.abs(V - V1).max() <= 5e-3
    assert np.linalg.eigvalsh(V).min() > 0 and np.linalg.eigvalsh(Mx).min() > 0


def test_p13_psd_equivalence():
    """M is positive semi-definite iff V is, whenever Cbar > 2/5 (Schur
    complement, then the congruence W = Q^T X Q = diag(Cbar, V)); checked on
    perturbations that grow until f takes negative values."""
    n, L = 24, 8.0
    rng = np.random.default_rng(13)
    seen = {True: 0, False: 0}
    for amp in (0.05, 0.3, 0.8, 1.5, 3.0, 6.0):
        for _ in range(6):
            q = amp * rng.normal(size=3)
            t = amp * rng.normal(size=(3, 3))
            t = 0.5 * (t + t.T)
            t -= np.trace(t) / 3 * np.eye(3)
            f = _thirteen_moment(n, L, 1.0, np.zeros(3), 1.0, q, t)
            Mx = kinetic.realizability_matrix(f, n, L)
            C, V = kinetic.reduced_realizability(Mx)
            if not C > 0.4:
                continue
            psd_m = np.linalg.eigvalsh(Mx).min() >= -1e-12
            psd_v = np.linalg.eigvalsh(V).min() >= -1e-12
            assert psd_m == psd_v, (amp, np.linalg.eigvalsh(Mx), np.linalg.eigvalsh(V))
            seen[psd_m] += 1
    assert seen[True] > 0 and seen[False] > 0, seen
