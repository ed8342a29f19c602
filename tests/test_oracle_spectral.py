"""Pins of the FP64 collision oracle against facts fixed by the paper and by
mathematics, each independent of the oracle's own code path.

  P1  naive separable DFT  vs numpy.fft with the grid phase (-1)^ktilde
  P2  phi_R / psi_R closed forms vs quadrature of their defining integrals
  P3  fast (product-in-v) evaluation vs the classic O(n^2) sum over l+m=k
  P5  Q(M, M) = 0 for Maxwellians (hypothesis (H3))
  P6  mass conserved before projection; all five invariants after (H1)
  P7  BKW exact solution for the gamma = 0 kernel: amplitude = C 4 pi / 15
  P8  hard-sphere loss rate of a Maxwellian, 4 pi int |v - v*| M dv*
  P9  direct (v*, sigma) quadrature of the Boltzmann integral (Sec. 2.1)
  P10 translation and reflection equivariance on the periodic grid
"""
import math

import numpy as np
import pytest
import scipy.integrate as si
from scipy.special import erf

import bz_inputs as gen
from oracle import directions, spectral


def make_plan(n=16, L=8.0, R=None, gamma=1.0, c=4.0, rule=("icosa6",)):
    if rule[0] == "icosa6":
        d, w = directions.icosa6()
    elif rule[0] == "spiral":
        d, w = directions.spiral(rule[1])
    else:
        d, w = directions.product(rule[1], rule[2])
    return spectral.Plan(n, L, spectral.default_R(L) if R is None else R, gamma, c, d, w)


# ---------------------------------------------------------------- P1
@pytest.mark.parametrize("n", [8, 12, 16])
def test_p1_dft_matches_numpy_fft(n):
    L = 5.0
    rng = np.random.default_rng(n)
    f = rng.normal(size=(n, n, n))
    fh = spectral.forward(f, n, L)
    k = np.arange(n)
    kt = np.where(k < n // 2, k, k - n)
    sign = (-1.0) ** (kt[:, None, None] + kt[None, :, None] + kt[None, None, :])
    ref = sign * np.fft.fftn(f) / n ** 3
    ref[spectral.nyquist_mask(n)] = 0
    assert np.abs(fh - ref).max() <= 1e-14 * np.abs(ref).max()
    g = rng.normal(size=(n, n, n)) + 1j * rng.normal(size=(n, n, n))
    inv = spectral.inverse(g, n, L)
    ref_inv = np.fft.ifftn(sign * g) * n ** 3
    assert np.abs(inv - ref_inv).max() <= 1e-13 * np.abs(ref_inv).max()


# ---------------------------------------------------------------- P2
@pytest.mark.parametrize("gamma", [0.0, 0.5, 1.0])
def test_p2_phi_against_defining_integral(gamma):
    R = 3.3
    s = np.array([0.0, 0.37, 1.9, 4.4, 11.0])
    got = spectral.phi(s, R, gamma)
    for si_, g in zip(s, got):
        # phi_R(s) = int_{-R}^{R} |rho| a(|rho|) exp(i rho s) d rho, a = rho^(gamma-1)
        # asked to 1e-13 absolute, a tenth of the bound checked below (1e-14 is
        # below the rounding of the integrand's cancellation and quad warns)
        val, _ = si.quad(lambda r: 2.0 * r ** gamma * math.cos(r * si_), 0.0, R,
                         limit=400, epsabs=1e-13, epsrel=1e-13)
        assert abs(g - val) <= 1e-12 * max(1.0, abs(val)), (gamma, si_, g, val)


@pytest.mark.parametrize("gamma", [0.0, 1.0])
def test_p2_phi_quadrature_matches_closed_form(gamma):
    R = spectral.max_R(8.0)
    s = np.linspace(0.0, 18.0, 301)
    a = spectral.phi(s, R, gamma)
    b = spectral.phi_quadrature(s, R, gamma)
    assert np.abs(a - b).max() <= 1e-12 * np.abs(a).max()


def test_p2_psi_is_disc_integral():
    R = 3.3
    for r in [0.0, 0.5, 2.0, 7.3]:
        # int over the disc |y| <= R of exp(i m.y) dy with |m| = r (polar form)
        # asked to 1e-11, a tenth of the bound checked below (tighter requests
        # are below the rounding of the inner integral and dblquad warns)
        val, _ = si.dblquad(lambda th, rho: rho * math.cos(rho * r * math.cos(th)),
                            0.0, R, 0.0, 2.0 * math.pi, epsabs=1e-11, epsrel=1e-11)
        got = spectral.psi(np.array([r]), R)[0]
        assert abs(got - val) <= 1e-10 * max(1.0, abs(val)), (r, got, val)


def test_loss_multiplier_at_zero_mode():
    """Bhat_M(0) = sum w_p phi(0) psi(0) = 2 pi * R^2 * pi R^2 for hard spheres,
    equal to the exact int int_{B_R^2} delta(x.y) dx dy = 2 pi^2 R^4."""
    for rule in [("icosa6",), ("spiral", 32), ("product", 4, 4)]:
        p = make_plan(n=8, rule=rule)
        b = spectral.bhat_m(p)
        assert abs(b[0, 0, 0] - 2 * math.pi ** 2 * p.R ** 4) <= 1e-12 * b[0, 0, 0]


def test_direction_rules():
    for d, w, m in [directions.icosa6() + (6,), directions.spiral(32) + (32,),
                    directions.product(4, 4) + (16,)]:
        assert d.shape == (m, 3) and w.shape == (m,)
        assert abs(w.sum() - 2 * math.pi) <= 1e-13
        assert np.abs(np.linalg.norm(d, axis=1) - 1).max() <= 1e-15
    # the six icosahedral axes integrate every even polynomial of degree <= 4
    # exactly over the half sphere: mean of (e.a)^2 = 1/3, (e.a)^4 = 1/5
    d, w = directions.icosa6()
    a = np.array([0.3, -0.5, 0.81])
    a /= np.linalg.norm(a)
    c = d @ a
    assert abs((w * c ** 2).sum() / (2 * math.pi) - 1 / 3) <= 1e-14
    assert abs((w * c ** 4).sum() / (2 * math.pi) - 1 / 5) <= 1e-14


# ---------------------------------------------------------------- P3
def brute_force_q(f, plan):
    """Classic spectral sum Qhat_k = sum_{l+m=k (mod n)} fhat_l fhat_m beta(l,m),
    beta(l,m) = sum_p w_p alpha_p(l) alpha'_p(m) - Bhat_M(m), O(n^2)."""
    n = plan.n
    fh = spectral.forward(f, n, plan.L)
    al = np.stack([spectral.multipliers(plan, p)[0] for p in range(plan.m)])
    ap = np.stack([spectral.multipliers(plan, p)[1] for p in range(plan.m)])
    bm = (plan.weights[:, None, None, None] * al * ap).sum(0)
    qh = np.zeros((n, n, n), dtype=complex)
    for l1 in range(n):
        for l2 in range(n):
            for l3 in range(n):
                if fh[l1, l2, l3] == 0:
                    continue
                beta = np.tensordot(plan.weights * al[:, l1, l2, l3], ap, axes=(0, 0)) - bm
                g = fh * beta
                qh += fh[l1, l2, l3] * np.roll(g, (l1, l2, l3), axis=(0, 1, 2))
    return plan.kernel_c * spectral.inverse(qh, n, plan.L)


@pytest.mark.parametrize("n,gamma", [(8, 1.0), (12, 1.0), (8, 0.5)])
def test_p3_fast_equals_classic_sum(n, gamma):
    plan = make_plan(n=n, L=6.0, gamma=gamma)
    rng = np.random.default_rng(3)
    f = gen.bimaxwellian_cell(n, 6.0, rng) + 0.01 * rng.uniform(size=(n, n, n))
    q = spectral.collide(f, plan)
    qb = brute_force_q(f, plan)
    assert np.abs(qb.imag).max() <= 1e-12 * np.abs(qb.real).max()
    assert np.linalg.norm(q - qb.real) <= 1e-12 * np.linalg.norm(qb.real)


# ---------------------------------------------------------------- P5, P6
def test_p5_maxwellian_is_equilibrium():
    plan = make_plan(n=32, L=8.0, rule=("spiral", 32))
    f = gen.maxwellian(32, 8.0, 1.0, [0.3, -0.2, 0.1], 1.0)
    q, qp, ql = spectral.collide_parts(f, plan)
    assert np.linalg.norm(q) <= 1e-8 * np.linalg.norm(qp)


def test_p5_q_is_not_trivially_zero():
    plan = make_plan(n=16)
    f = gen.bimaxwellian_cell(16, 8.0, np.random.default_rng(1))
    q, qp, ql = spectral.collide_parts(f, plan)
    assert np.linalg.norm(q) >= 0.05 * np.linalg.norm(qp)


def test_p6_conservation():
    n, L = 16, 8.0
    plan = make_plan(n=n, L=L)
    f = gen.bimaxwellian_cell(n, L, np.random.default_rng(7))
    q = spectral.collide(f, plan)
    # mass is exact before projection: alpha, alpha' are even
    assert abs(q.sum()) <= 1e-13 * np.abs(q).sum()
    qp = spectral.project(q, n, L)
    assert spectral.moment_drift(qp, n, L) <= 1e-13
    # the projection is the minimum-norm correction: Q - Qp lies in range(C^T)
    C = spectral.moment_matrix(n, L)
    resid = (q - qp).ravel()
    coef, *_ = np.linalg.lstsq(C.T, resid, rcond=None)
    assert np.linalg.norm(C.T @ coef - resid) <= 1e-13 * np.linalg.norm(q)


# ---------------------------------------------------------------- P7
def test_p7_bkw_rate_and_shape():
    """For the gamma = 0 kernel Btilde = C/|x| the sigma-form kernel is
    B = (C/4)/cos(theta/2); the BKW profile decays as dK/dt = lambda (1-K)
    with lambda = (1/4) int_{S^2} B (1 - cos^2 theta) d sigma = C 4 pi / 15."""
    n, L = 32, 8.0
    plan = make_plan(n=n, L=L, R=spectral.max_R(L), gamma=0.0, rule=("spiral", 32))
    K = 0.7
    f = gen.bkw_profile(n, L, K)
    h = 1e-5
    dK = (gen.bkw_profile(n, L, K + h) - gen.bkw_profile(n, L, K - h)) / (2 * h)
    g = (1 - K) * dK
    q = spectral.collide(f, plan)
    amp = (q * g).sum() / (g * g).sum()
    lam = plan.kernel_c * 4 * math.pi / 15
    assert abs(amp / lam - 1) <= 1e-5, amp / lam
    assert np.linalg.norm(q - amp * g) / np.linalg.norm(amp * g) <= 0.02


# ---------------------------------------------------------------- P8
def test_p8_hard_sphere_loss_rate():
    n, L = 32, 8.0
    plan = make_plan(n=n, L=L, R=spectral.max_R(L), rule=("spiral", 256))
    f = gen.maxwellian(n, L, 1.0, [0, 0, 0], 1.0)
    lam = spectral.inverse(spectral.bhat_m(plan) * spectral.forward(f, n, L), n, L).real
    loss = plan.kernel_c * lam
    v = spectral.velocity_nodes(n, L)
    c = np.sqrt(v[:, None, None] ** 2 + v[None, :, None] ** 2 + v[None, None, :] ** 2)
    s = np.maximum(c / math.sqrt(2.0), 1e-12)
    exact = 4 * math.pi * math.sqrt(2.0) * ((s + 1 / (2 * s)) * erf(s) + np.exp(-s * s) / math.sqrt(math.pi))
    # loss term f * rate: the truncation |x|,|y| <= R only matters where f is small
    assert np.abs(f * (loss - exact)).max() <= 1e-3 * np.abs(f * exact).max()
    fit = (f * loss * f * exact).sum() / ((f * exact) ** 2).sum()
    assert abs(fit - 1.0) <= 1e-5


# ---------------------------------------------------------------- P9
@pytest.mark.slow
def test_p9_direct_sigma_quadrature():
    """Q(f,f)(v) = int int |v - v*| [f(v') f(v*') - f(v) f(v*)] d sigma dv*
    (hard spheres) by brute-force quadrature, at a few grid points."""
    n, L = 32, 8.0
    plan = make_plan(n=n, L=L, R=spectral.max_R(L), rule=("spiral", 128))
    comps = [(0.7, np.array([0.6, 0.0, -0.2]), 0.8), (0.5, np.array([-0.8, 0.4, 0.3]), 1.2)]

    def fan(x):
        out = 0.0
        for rho, u, T in comps:
            out = out + rho / (2 * math.pi * T) ** 1.5 * np.exp(-((x - u) ** 2).sum(-1) / (2 * T))
        return out
    v = spectral.velocity_nodes(n, L)
    V = np.stack(np.meshgrid(v, v, v, indexing="ij"), -1)
    q = spectral.collide(fan(V), plan)
    xg, wg = np.polynomial.legendre.leggauss(36)
    a = 7.0
    g1 = a * xg
    w1 = a * wg
    VS = np.stack(np.meshgrid(g1, g1, g1, indexing="ij"), -1).reshape(-1, 3)
    WS = (w1[:, None, None] * w1[None, :, None] * w1[None, None, :]).ravel()
    ct, wct = np.polynomial.legendre.leggauss(24)
    ph = np.arange(48) * 2 * math.pi / 48
    CT, PH = np.meshgrid(ct, ph, indexing="ij")
    ST = np.sqrt(1 - CT ** 2)
    SIG = np.stack([ST * np.cos(PH), ST * np.sin(PH), CT], -1).reshape(-1, 3)
    WSIG = np.repeat(wct, 48) * (2 * math.pi / 48)
    fvs = fan(VS)
    for (i, j, k) in [(16, 16, 16), (18, 15, 16), (13, 17, 19), (20, 16, 12)]:
        vv = V[i, j, k]
        qrel = vv[None, :] - VS
        g = np.linalg.norm(qrel, axis=1)
        mid = 0.5 * (vv[None, :] + VS)
        gain = 0.0
        for s0 in range(0, SIG.shape[0], 128):
            sg = SIG[s0:s0 + 128]
            vp = mid[:, None, :] + 0.5 * g[:, None, None] * sg[None]
            vps = mid[:, None, :] - 0.5 * g[:, None, None] * sg[None]
            gain += ((fan(vp) * fan(vps)) @ WSIG[s0:s0 + 128] * g * WS).sum()
        loss = fan(vv) * (g * fvs * WS).sum() * 4 * math.pi
        ref = gain - loss
        scale = loss
        assert abs(q[i, j, k] - ref) <= 2e-3 * scale, (i, j, k, q[i, j, k], ref)


# ---------------------------------------------------------------- P10
def test_p10_equivariance():
    n, L = 16, 8.0
    plan = make_plan(n=n, L=L)
    rng = np.random.default_rng(11)
    f = gen.bimaxwellian_cell(n, L, rng)
    q = spectral.collide(f, plan)
    sh = (3, -2, 5)
    qs = spectral.collide(np.roll(f, sh, axis=(0, 1, 2)), plan)
    assert np.abs(qs - np.roll(q, sh, axis=(0, 1, 2))).max() <= 1e-13 * np.abs(q).max()
    refl = (-np.arange(n)) % n
    fr = f[refl][:, refl][:, :, refl]
    qr = spectral.collide(fr, plan)
    assert np.abs(qr - q[refl][:, refl][:, :, refl]).max() <= 1e-13 * np.abs(q).max()


def test_rel_err_floor():
    q = np.ones(8)
    assert spectral.rel_err(q * (1 + 1e-6), q) == pytest.approx(1e-6, rel=1e-6)
    small = q * 1e-6
    assert spectral.rel_err(small + 1e-3, small, loss_ref=q) == pytest.approx(1e-3 / 0.05, rel=1e-9)


def test_fft_mode_equals_the_naive_dft_oracle():
    # the library-FFT evaluation is the same discrete operator (phases cancel in pairs)
    import bz_inputs as gen
    from oracle import directions
    for n, rule in ((16, directions.icosa6()), (24, directions.spiral(32))):
        plan = spectral.Plan(n, 8.0, spectral.default_R(8.0), 1.0, 4.0, *rule)
        f = gen.shock_batch(1, n, 8.0, seed=3)[0]
        q = spectral.collide(f, plan)
        assert np.abs(spectral.collide_fft(f, plan) - q).max() <= 1e-12 * np.abs(q).max()
        parts, ref_parts = spectral.collide_fft(f, plan, parts=True), spectral.collide_parts(f, plan)
        for a, b in zip(parts, ref_parts):
            assert np.abs(a - b).max() <= 1e-12 * np.abs(b).max()


# ---------------------------------------------------------------- dealiased variant
def brute_force_q_nowrap(f, plan):
    """Classic spectral sum over l + m = k as integers (no wrap-around), l, m
    among the truncated series' modes, for the output modes |ktilde| < n/2."""
    n = plan.n
    fh = spectral.forward(f, n, plan.L)
    al = np.stack([spectral.multipliers(plan, p)[0] for p in range(plan.m)])
    ap = np.stack([spectral.multipliers(plan, p)[1] for p in range(plan.m)])
    bm = (plan.weights[:, None, None, None] * al * ap).sum(0)
    kt = np.where(np.arange(n) < n // 2, np.arange(n), np.arange(n) - n)
    band = np.flatnonzero(np.abs(kt) < n // 2)
    big = np.zeros((2 * n,) * 3, dtype=complex)  # index ktilde + n
    for l1 in band:
        for l2 in band:
            for l3 in band:
                if fh[l1, l2, l3] == 0:
                    continue
                beta = np.tensordot(plan.weights * al[:, l1, l2, l3], ap, axes=(0, 0)) - bm
                g = fh * beta
                for m1 in band:
                    for m2 in band:
                        k = (kt[l1] + kt[m1] + n, kt[l2] + kt[m2] + n)
                        big[k[0], k[1], kt[l3] + kt[band] + n] += fh[l1, l2, l3] * g[m1, m2, band]
    qh = np.zeros((n, n, n), dtype=complex)
    for a in band:
        for b in band:
            qh[a, b, band] = big[kt[a] + n, kt[b] + n, kt[band] + n]
    return plan.kernel_c * spectral.inverse(qh, n, plan.L)


@pytest.mark.parametrize("n", [8, 12])
def test_dealiased_equals_nonperiodic_sum(n):
    plan = make_plan(n=n, L=6.0, gamma=1.0)
    rng = np.random.default_rng(4)
    f = gen.bimaxwellian_cell(n, 6.0, rng) + 0.01 * rng.uniform(size=(n, n, n))
    q = spectral.collide_dealiased(f, plan)
    qb = brute_force_q_nowrap(f, plan)
    assert np.abs(qb.imag).max() <= 1e-12 * np.abs(qb.real).max()
    assert np.linalg.norm(q - qb.real) <= 1e-12 * np.linalg.norm(qb.real)
    # and it differs from the circular (aliased) sum by the wrapped terms
    assert np.linalg.norm(q - spectral.collide(f, plan)) > 1e-8 * np.linalg.norm(q)


def test_dealiased_close_to_aliased_for_resolved_f():
    # a well-resolved distribution has little energy near the band edge: the two agree closely
    import bz_inputs
    plan = make_plan(n=16, L=8.0, gamma=1.0)
    f = bz_inputs.maxwellian(16, 8.0, 1.0, [0.2, -0.1, 0.0], 1.5)
    q, qa = spectral.collide_dealiased(f, plan), spectral.collide(f, plan)
    assert np.linalg.norm(q - qa) <= 1e-3 * np.linalg.norm(spectral.collide_parts(f, plan)[1])
