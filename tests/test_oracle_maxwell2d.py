"""Pins of the 2D Maxwell-molecule oracle (Sec. 4.4.1, the 2d case) against
facts fixed by mathematics, each independent of the oracle's own code path.

  D1  naive separable 2D DFT vs numpy.fft with the grid phase (-1)^ktilde
  D2  fast (product-in-v) evaluation vs the classic O(n^2) sum over l+m=k
  D3  Q(M, M) = 0 for Maxwellians
  D4  mass conserved before projection; the four invariants after
  D5  exact relaxation of the traceless second moments of Maxwell molecules:
      int Q (v1^2 - v2^2) dv = -(pi C rho / 2) int f ((v1-u1)^2 - (v2-u2)^2) dv
      and the same for v1 v2 (any f; the Carleman kernel Btilde = C is the
      sigma-form kernel B = C/2 in two dimensions)
  D6  direct (v*, sigma) quadrature of the 2D Boltzmann integral
"""
import math

import numpy as np
import pytest

import bz_inputs as gen
from oracle import maxwell2d as m2, spectral


def test_d1_dft_matches_numpy_fft():
    n, L = 12, 5.0
    rng = np.random.default_rng(1)
    f = rng.normal(size=(n, n))
    fh = m2.forward(f, n, L)
    k = np.arange(n)
    kt = np.where(k < n // 2, k, k - n)
    sign = (-1.0) ** (kt[:, None] + kt[None, :])
    ref = sign * np.fft.fft2(f) / n ** 2
    ref[m2.nyquist_mask(n)] = 0
    assert np.abs(fh - ref).max() <= 1e-14 * np.abs(ref).max()
    g = rng.normal(size=(n, n)) + 1j * rng.normal(size=(n, n))
    assert np.abs(m2.inverse(g, n, L) - np.fft.ifft2(sign * g) * n ** 2).max() <= 1e-13 * np.abs(g).sum()


def brute_force_q(f, plan):
    """Qhat_k = C sum_{l+m=k (mod n)} fhat_l fhat_m (Bhat_F(l,m) - Bhat_F(m,m)),
    Bhat_F(l,m) = (pi/A) sum_p phi(l . e_p) phi(m . e_p'), term by term."""
    n, L, R = plan.n, plan.L, plan.R
    fh = m2.forward(f, n, L)
    k = spectral.wavenumbers(n, L)
    th = math.pi * np.arange(1, plan.A + 1) / plan.A
    sinc = lambda x: np.where(np.abs(x) < 1e-300, 1.0, np.sin(x) / np.where(x == 0, 1.0, x))
    ph = lambda s: 2 * R * sinc(R * s)
    qh = np.zeros((n, n), dtype=complex)
    for l1 in range(n):
        for l2 in range(n):
            if fh[l1, l2] == 0:
                continue
            for m1 in range(n):
                for m2_ in range(n):
                    if fh[m1, m2_] == 0:
                        continue
                    bl = bm = 0.0
                    for t in th:
                        c, s = math.cos(t), math.sin(t)
                        pm = ph(-k[m1] * s + k[m2_] * c)
                        bl += ph(k[l1] * c + k[l2] * s) * pm
                        bm += ph(k[m1] * c + k[m2_] * s) * pm
                    beta = (math.pi / plan.A) * (bl - bm)
                    qh[(l1 + m1) % n, (l2 + m2_) % n] += fh[l1, l2] * fh[m1, m2_] * beta
    return plan.kernel_c * m2.inverse(qh, n, L)


@pytest.mark.parametrize("n,A", [(8, 6), (12, 5)])
def test_d2_fast_equals_classic_sum(n, A):
    plan = m2.make_plan(n, L=6.0, A=A, kernel_c=1.3)
    rng = np.random.default_rng(n)
    f = gen.bimaxwellian2d_batch(1, n, 6.0, seed=n)[0] + 0.01 * rng.uniform(size=(n, n))
    q = m2.collide(f, plan)
    qb = brute_force_q(f, plan)
    assert np.abs(qb.imag).max() <= 1e-12 * np.abs(qb.real).max()
    assert np.linalg.norm(q - qb.real) <= 1e-12 * np.linalg.norm(qb.real)


def test_d3_maxwellian_is_equilibrium():
    n, L = 32, 8.0
    plan = m2.make_plan(n, L, A=32)  # default R; at the largest R periodisation leaves ~3e-6
    f = gen.maxwellian2d(n, L, 1.0, [0.3, -0.2], 1.0)
    q, qp, ql = m2.collide_parts(f, plan)
    assert np.linalg.norm(q) <= 1e-8 * np.linalg.norm(qp)
    g = gen.bimaxwellian2d_batch(1, n, L, seed=3)[0]
    q, qp, ql = m2.collide_parts(g, plan)
    assert np.linalg.norm(q) >= 0.05 * np.linalg.norm(qp)  # not trivially zero


def test_d4_conservation():
    n, L = 32, 8.0
    plan = m2.make_plan(n, L, A=16)
    f = gen.bimaxwellian2d_batch(1, n, L, seed=4)[0]
    q = m2.collide(f, plan)
    assert abs(q.sum()) <= 1e-13 * np.abs(q).sum()  # alpha, alpha' even: mass is exact
    qp = m2.project(q, n, L)
    assert m2.moment_drift(qp, n, L) <= 1e-13
    C = m2.moment_matrix(n, L)
    resid = (q - qp).ravel()
    coef, *_ = np.linalg.lstsq(C.T, resid, rcond=None)
    assert np.linalg.norm(C.T @ coef - resid) <= 1e-13 * np.linalg.norm(q)


@pytest.mark.parametrize("c", [1.0, 2.5])
def test_d5_second_moment_relaxation_rate(c):
    # the truncation |x|, |y| <= R drops the rare far collisions: with R the
    # largest radius free of period overlap the identity holds to 1.4e-3 at
    # L = 8, 3e-5 at L = 10 and 3e-7 at L = 12
    n, L = 64, 12.0
    plan = m2.make_plan(n, L, R=spectral.max_R(L), A=32, kernel_c=c)
    u = np.array([0.4, -0.3])
    f = gen.gaussian2d(n, L, 1.2, u, 0.7, 1.6, 0.6)
    v = spectral.velocity_nodes(n, L)
    V1, V2 = np.meshgrid(v, v, indexing="ij")
    dv2 = (2 * L / n) ** 2
    rho = f.sum() * dv2
    q = m2.collide(f, plan)
    rate = -math.pi * c * rho / 2
    for phi_q, phi_c in [(V1 ** 2 - V2 ** 2, (V1 - u[0]) ** 2 - (V2 - u[1]) ** 2),
                         (V1 * V2, (V1 - u[0]) * (V2 - u[1]))]:
        lhs = (q * phi_q).sum() * dv2
        rhs = rate * (f * phi_c).sum() * dv2
        assert abs(lhs / rhs - 1) <= 1e-6, (lhs, rhs)


def test_d6_direct_sigma_quadrature():
    """Q(v) = int_{R^2} int_{S^1} (C/2) [f(v') f(v*') - f(v) f(v*)] d sigma dv*,
    v' = (v + v*)/2 + |v - v*| sigma / 2, v*' = (v + v*)/2 - |v - v*| sigma / 2,
    by brute-force quadrature at a few grid points."""
    n, L, c = 32, 8.0, 1.0
    plan = m2.make_plan(n, L, R=spectral.max_R(L), A=64, kernel_c=c)
    comps = [(0.7, np.array([0.6, -0.2]), 0.8), (0.5, np.array([-0.8, 0.4]), 1.3)]

    def fan(x):
        out = 0.0
        for rho, uu, T in comps:
            out = out + rho / (2 * math.pi * T) * np.exp(-((x - uu) ** 2).sum(-1) / (2 * T))
        return out
    v = spectral.velocity_nodes(n, L)
    V = np.stack(np.meshgrid(v, v, indexing="ij"), -1)
    q = m2.collide(fan(V), plan)
    xg, wg = np.polynomial.legendre.leggauss(64)
    a = 7.5
    g1, w1 = a * xg, a * wg
    VS = np.stack(np.meshgrid(g1, g1, indexing="ij"), -1).reshape(-1, 2)
    WS = (w1[:, None] * w1[None, :]).ravel()
    ang = np.arange(96) * 2 * math.pi / 96
    SIG = np.stack([np.cos(ang), np.sin(ang)], -1)
    wsig = 2 * math.pi / 96
    fvs = fan(VS)
    for (i, j) in [(16, 16), (18, 15), (13, 19), (20, 12)]:
        vv = V[i, j]
        g = np.linalg.norm(vv[None, :] - VS, axis=1)
        mid = 0.5 * (vv[None, :] + VS)
        vp = mid[:, None, :] + 0.5 * g[:, None, None] * SIG[None]
        vps = mid[:, None, :] - 0.5 * g[:, None, None] * SIG[None]
        gain = (c / 2) * ((fan(vp) * fan(vps)).sum(1) * wsig * WS).sum()
        loss = (c / 2) * fan(vv) * (fvs * WS).sum() * 2 * math.pi
        assert abs(q[i, j] - (gain - loss)) <= 1e-4 * loss, (i, j, q[i, j], gain - loss)
