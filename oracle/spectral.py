"""FP64 oracle of the fast spectral collision operator (Sec. 4.4.1).

TEST INFRASTRUCTURE ONLY (see package doc).

What is computed, per spatial cell, for a distribution f sampled on the
velocity grid v_j = (j - N/2) dv, dv = 2L/N, j in [0,N)^3 (Sec. 4.1):

  1. Fourier coefficients of the periodised f on [-L, L)^3 (Sec. 4.4.1,
     truncated Fourier series), approximated by the grid quadrature
        fhat_k = N^-3 sum_j f_j exp(-i kappa_k . v_j),
     kappa_k = (pi/L) ktilde, ktilde in [-N/2, N/2)^3.  The Nyquist modes
     (any ktilde_i = -N/2) are set to zero so that the truncated series is
     symmetric in k, as the paper's k = -N..N sums are.
  2. The truncated Carleman operator Q^R (Sec. 4.4.1) with the decoupled kernel
     Btilde(x, y) = C a(|x|) b(|y|), a(r) = r^(gamma-1), b = 1
     (gamma = 1 is the hard-sphere kernel B = |v - v*| with C = 4).
     Writing x = rho e (e on the half sphere) turns the spectral kernel
     Bhat_F(l, m) into a half-sphere integral of the product
        phi_R(l . e) * psi_R(|m - (m . e) e|),
        phi_R(s) = int_{-R}^{R} |rho| a(|rho|) exp(i rho s) d rho
                 = 2 int_0^R rho^gamma cos(rho s) d rho,
        psi_R(r) = int over the disc |y| <= R in the plane normal to e of
                   exp(i m . y) dy = 2 pi R J1(R r) / r   (pi R^2 at r = 0).
     A direction rule (e_p, w_p), sum w_p = 2 pi, turns it into the sum of
     products alpha_p(l) alpha'_p(m) of the fast method (equation for
     beta_F as a sum over A directions).
  3. Gain: for each direction, the two inverse transforms
        A_p  = sum_k alpha_p(k)  fhat_k exp(i kappa_k . v_j),
        A'_p = sum_k alpha'_p(k) fhat_k exp(i kappa_k . v_j),
     are real, and Q+_j = sum_p w_p A_p,j A'_p,j (one discrete convolution
     per direction).
  4. Loss: with the same quadrature, Bhat_M(k) = sum_p w_p alpha_p(k)
     alpha'_p(k) gives Lambda_j = sum_k Bhat_M(k) fhat_k exp(i kappa_k . v_j),
     and the loss is fN_j Lambda_j, fN = sum_k fhat_k exp(i kappa_k . v_j)
     the truncated series itself (the beta = Bhat(l,m) - Bhat(m,m) split of
     the sum over l + m = k, in which both factors are fhat).
  5. Q_j = C (Q+_j - fN_j Lambda_j).

Transforms are separable naive DFTs (an n x n matrix per axis); the only
library routines used are a matrix product (tensordot), the Bessel function
J1, Gauss-Legendre nodes, and a 5x5 linear solve.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np
import scipy.special as sps

GL_NODES = 256


@dataclass
class Plan:
    """Operator parameters: grid (n, L), truncation R, kernel exponent gamma,
    kernel constant C, direction rule (dirs, weights)."""
    n: int
    L: float
    R: float
    gamma: float
    kernel_c: float
    dirs: np.ndarray
    weights: np.ndarray
    _cache: dict = field(default_factory=dict, repr=False)

    @property
    def m(self) -> int:
        return len(self.weights)


def default_R(L: float) -> float:
    """Default truncation radius (sqrt(2) - 1) L, the value 3.3 the paper
    prints for L = 8 in every test of Sec. 5."""
    return (math.sqrt(2.0) - 1.0) * L


def max_R(L: float) -> float:
    """Largest radius free of period overlap, T >= (3 + sqrt 2) S / 2 with
    R = 2S (Sec. 4.4.1): R = 4 L / (3 + sqrt 2)."""
    return 4.0 * L / (3.0 + math.sqrt(2.0))


def velocity_nodes(n: int, L: float) -> np.ndarray:
    return (np.arange(n, dtype=np.float64) - n // 2) * (2.0 * L / n)


def wavenumbers(n: int, L: float) -> np.ndarray:
    """kappa_k = (pi / L) ktilde with ktilde = k (k < n/2) or k - n."""
    k = np.arange(n)
    kt = np.where(k < n // 2, k, k - n).astype(np.float64)
    return (math.pi / L) * kt


def nyquist_mask(n: int) -> np.ndarray:
    nyq = np.arange(n) == n // 2
    return nyq[:, None, None] | nyq[None, :, None] | nyq[None, None, :]


def _along(mat: np.ndarray, x: np.ndarray, axis: int) -> np.ndarray:
    return np.moveaxis(np.tensordot(mat, x, axes=([1], [axis])), 0, axis)


def forward(f: np.ndarray, n: int, L: float) -> np.ndarray:
    """fhat_k = n^-3 sum_j f_j exp(-i kappa_k . v_j), Nyquist modes zeroed."""
    E = np.exp(-1j * np.outer(wavenumbers(n, L), velocity_nodes(n, L)))
    g = f.astype(np.complex128)
    for ax in range(3):
        g = _along(E, g, ax)
    g = g / float(n) ** 3
    g[nyquist_mask(n)] = 0.0
    return g


def inverse(g: np.ndarray, n: int, L: float) -> np.ndarray:
    """sum_k g_k exp(i kappa_k . v_j) on the grid."""
    E = np.exp(1j * np.outer(velocity_nodes(n, L), wavenumbers(n, L)))
    y = g
    for ax in range(3):
        y = _along(E, y, ax)
    return y


def phi(s, R: float, gamma: float) -> np.ndarray:
    """phi_R(s) = 2 int_0^R rho^gamma cos(rho s) d rho.

    gamma = 1: R^2 [2 sinc(Rs) - sinc(Rs/2)^2]; gamma = 0: 2R sinc(Rs)
    (sinc x = sin x / x); otherwise Gauss-Legendre after rho = R t^2."""
    s = np.asarray(s, dtype=np.float64)
    if gamma == 1.0:
        return R * R * (2.0 * np.sinc(R * s / math.pi) - np.sinc(R * s / (2.0 * math.pi)) ** 2)
    if gamma == 0.0:
        return 2.0 * R * np.sinc(R * s / math.pi)
    return phi_quadrature(s, R, gamma)


def phi_quadrature(s, R: float, gamma: float, nodes: int = GL_NODES) -> np.ndarray:
    """phi_R by quadrature: rho = R t^2 gives
    4 R^(gamma+1) int_0^1 t^(2 gamma + 1) cos(R s t^2) dt."""
    s = np.asarray(s, dtype=np.float64)
    x, w = np.polynomial.legendre.leggauss(nodes)
    t = 0.5 * (x + 1.0)
    wt = 0.5 * w * t ** (2.0 * gamma + 1.0)
    flat = s.ravel()
    out = np.empty_like(flat)
    chunk = 8192
    for i in range(0, flat.size, chunk):
        c = flat[i:i + chunk]
        out[i:i + chunk] = np.cos(R * c[:, None] * (t * t)[None, :]) @ wt
    return (4.0 * R ** (gamma + 1.0) * out).reshape(s.shape)


def psi(r, R: float) -> np.ndarray:
    """psi_R(r) = 2 pi R J1(R r) / r, with the limit pi R^2 at r = 0."""
    r = np.asarray(r, dtype=np.float64)
    out = np.full(r.shape, math.pi * R * R)
    nz = r > 0.0
    out[nz] = 2.0 * math.pi * R * sps.j1(R * r[nz]) / r[nz]
    return out


def multipliers(plan: Plan, p: int):
    """alpha_p(k) = phi_R(kappa_k . e_p), alpha'_p(k) = psi_R(|kappa_k -
    (kappa_k . e_p) e_p|) on the [k1][k2][k3] grid."""
    key = ("mult", p)
    if key in plan._cache:
        return plan._cache[key]
    kap = wavenumbers(plan.n, plan.L)
    K1, K2, K3 = np.meshgrid(kap, kap, kap, indexing="ij")
    e = plan.dirs[p]
    s = K1 * e[0] + K2 * e[1] + K3 * e[2]
    P1 = K1 - s * e[0]
    P2 = K2 - s * e[1]
    P3 = K3 - s * e[2]
    r = np.sqrt(P1 * P1 + P2 * P2 + P3 * P3)
    res = (phi(s, plan.R, plan.gamma), psi(r, plan.R))
    if 16 * plan.n ** 3 * plan.m <= 1 << 29:  # keep all directions when they fit in 512 MiB
        plan._cache[key] = res
    return res


def bhat_m(plan: Plan) -> np.ndarray:
    """Bhat_M(k) = sum_p w_p alpha_p(k) alpha'_p(k) (the loss multiplier)."""
    if "bhat" in plan._cache:
        return plan._cache["bhat"]
    acc = np.zeros((plan.n,) * 3)
    for p in range(plan.m):
        a, ap = multipliers(plan, p)
        acc += plan.weights[p] * a * ap
    plan._cache["bhat"] = acc
    return acc


def collide_parts(f: np.ndarray, plan: Plan):
    """Return (Q, Qplus, loss) for one cell, all float64 [n][n][n], already
    multiplied by the kernel constant C.  Asserts that every inverse transform
    is real to 1e-12 of its magnitude."""
    n, L = plan.n, plan.L
    fh = forward(f, n, L)
    qplus = np.zeros((n, n, n))
    for p in range(plan.m):
        a, ap = multipliers(plan, p)
        A = inverse(a * fh, n, L)
        Ap = inverse(ap * fh, n, L)
        for Y in (A, Ap):
            assert np.abs(Y.imag).max() <= 1e-12 * max(np.abs(Y.real).max(), 1e-300)
        qplus += plan.weights[p] * A.real * Ap.real
    lam = inverse(bhat_m(plan) * fh, n, L)
    fn = inverse(fh, n, L)
    for Y in (lam, fn):
        assert np.abs(Y.imag).max() <= 1e-12 * max(np.abs(Y.real).max(), 1e-300)
    loss = fn.real * lam.real
    c = plan.kernel_c
    return c * (qplus - loss), c * qplus, c * loss


def collide(f: np.ndarray, plan: Plan) -> np.ndarray:
    return collide_parts(f, plan)[0]


def padded_plan(plan: Plan) -> Plan:
    """The same operator on the 3n/2 grid over the same box [-L, L)^3 (same
    wavenumber spacing pi/L, same R, kernel and directions)."""
    if (3 * plan.n) % 2:
        raise ValueError("n must be even")
    return Plan(3 * plan.n // 2, plan.L, plan.R, plan.gamma, plan.kernel_c, plan.dirs, plan.weights)


def _band(n: int) -> np.ndarray:
    """Indices (on an n-point wavenumber axis) of the modes |ktilde| < n/2."""
    k = np.arange(n)
    return np.where(k < n // 2, k, k - n)


def collide_dealiased(f: np.ndarray, plan: Plan, op=None) -> np.ndarray:
    """The truncated convolution without wrap-around: the sums over l + m = k
    taken over the truncated series' own modes, as integers (the paper's
    sums over l + m = k), for the output modes |ktilde| < n/2.  Evaluated by
    the 3/2 rule: the truncated series of f sampled on the 3n/2 grid, the fast
    operator there, and the result truncated back to the n modes (a product of
    two series with |ktilde| < n/2 has modes |ktilde| < n, and on a 3n/2-point
    axis the wrapped ones land outside |ktilde| < n/2).  `op` evaluates the
    operator on the padded grid (default collide; collide_fft is the same
    operator, pinned to it, and faster for large grids)."""
    n, L = plan.n, plan.L
    pp = padded_plan(plan)
    np_ = pp.n
    fh = forward(f, n, L)  # Nyquist zeroed
    kt = _band(n)
    sel = np.abs(kt) < n // 2
    ip = np.where(kt[sel] >= 0, kt[sel], kt[sel] + np_)  # the same modes on the padded axis
    g = np.zeros((np_,) * 3, dtype=complex)
    g[np.ix_(ip, ip, ip)] = fh[np.ix_(np.flatnonzero(sel), np.flatnonzero(sel), np.flatnonzero(sel))]
    fp = inverse(g, np_, L)
    assert np.abs(fp.imag).max() <= 1e-12 * np.abs(fp.real).max()
    qp = (op or collide)(fp.real, pp)
    qh = forward(qp, np_, L)
    out = np.zeros((n,) * 3, dtype=complex)
    out[np.ix_(np.flatnonzero(sel), np.flatnonzero(sel), np.flatnonzero(sel))] = qh[np.ix_(ip, ip, ip)]
    q = inverse(out, n, L)
    assert np.abs(q.imag).max() <= 1e-12 * np.abs(q.real).max()
    return q.real


def collide_fft(f: np.ndarray, plan: Plan, parts: bool = False):
    """The same operator with library FFTs for the transforms (the paper's CPU
    evaluation: an FFT per cell and direction).  On the grid v_j = (j - N/2) dv
    the exact transforms are the standard DFT times the phase (-1)^ktilde,
    which cancels between every forward/inverse pair, so
        A_p = N^3 IDFT(alpha_p DFT(f)/N^3), etc.
    Used to time a CPU evaluation whose cost scales like the method's; pinned
    to collide() in the tests."""
    n = plan.n
    fh = np.fft.fftn(f) / float(n) ** 3
    fh[nyquist_mask(n)] = 0.0

    def inv(g):
        return np.fft.ifftn(g).real * float(n) ** 3

    qplus = np.zeros((n, n, n))
    for p in range(plan.m):
        a, ap = multipliers(plan, p)
        qplus += plan.weights[p] * inv(a * fh) * inv(ap * fh)
    loss = inv(fh) * inv(bhat_m(plan) * fh)
    c = plan.kernel_c
    if parts:  # (Q, Q+, loss) as collide_parts returns them
        return c * (qplus - loss), c * qplus, c * loss
    return c * (qplus - loss)


def moment_matrix(n: int, L: float) -> np.ndarray:
    """C (5 x n^3): rows 1, v1, v2, v3, |v|^2 at the grid points (the
    collision invariants of hypothesis (H1); the common factor dv^3 cancels)."""
    v = velocity_nodes(n, L)
    V1, V2, V3 = np.meshgrid(v, v, v, indexing="ij")
    return np.stack([np.ones(n ** 3), V1.ravel(), V2.ravel(), V3.ravel(),
                     (V1 * V1 + V2 * V2 + V3 * V3).ravel()])


def project(q: np.ndarray, n: int, L: float) -> np.ndarray:
    """Least-squares projection onto {C Q = 0}: Q - C^T (C C^T)^-1 C Q.  The
    paper notes that periodisation loses the local invariants of (H1)
    (Sec. 2.1); this restores mass, momentum and energy exactly in FP64."""
    C = moment_matrix(n, L)
    G = C @ C.T
    lam = np.linalg.solve(G, C @ q.ravel())
    return (q.ravel() - C.T @ lam).reshape(q.shape)


def collide_batch(f: np.ndarray, plan: Plan, project_out: bool = True) -> np.ndarray:
    out = np.empty_like(f, dtype=np.float64)
    for c in range(f.shape[0]):
        q = collide(f[c], plan)
        out[c] = project(q, plan.n, plan.L) if project_out else q
    return out


def moment_drift(q: np.ndarray, n: int, L: float) -> float:
    """max_i |C_i Q| / sum_j |C_ij| |Q_j| over the five invariants."""
    C = moment_matrix(n, L)
    qq = q.ravel()
    return float(np.max(np.abs(C @ qq) / (np.abs(C) @ np.abs(qq))))


def rel_err(q_test: np.ndarray, q_ref: np.ndarray, loss_ref: np.ndarray | None = None) -> float:
    """Per-cell error ||dQ||_2 / max(||Q_ref||_2, 0.05 ||loss_ref||_2): the
    floor keeps near-equilibrium cells, whose Q is a small difference of
    gain and loss, from dividing by ~0."""
    den = np.linalg.norm(q_ref)
    if loss_ref is not None:
        den = max(den, 0.05 * np.linalg.norm(loss_ref))
    return float(np.linalg.norm(q_test - q_ref) / den)


def bhat_pair(lv, mv, R: float, gamma: float, dirs, weights) -> np.ndarray:
    """The direction rule's approximation of the spectral kernel Bhat(l, m):
    sum_p w_p phi_R(l . e_p) psi_R(|m - (m . e_p) e_p|) for wave vectors
    lv, mv [K, 3] (the sum over directions that replaces the half-sphere
    integral in Sec. 4.4.1, beta_F = sum_p alpha_p(l) alpha'_p(m))."""
    lv = np.atleast_2d(np.asarray(lv, dtype=np.float64))
    mv = np.atleast_2d(np.asarray(mv, dtype=np.float64))
    e = np.asarray(dirs, dtype=np.float64)
    s = lv @ e.T                                   # [K, P]
    me = mv @ e.T
    perp2 = (mv * mv).sum(axis=1)[:, None] - me * me
    r = np.sqrt(np.maximum(perp2, 0.0))
    return (phi(s, R, gamma) * psi(r, R)) @ np.asarray(weights, dtype=np.float64)


def hemisphere_gauss_rule(n_theta: int, n_phi: int):
    """Product rule on the half sphere z >= 0: Gauss-Legendre nodes in
    z = cos(theta) on [0, 1] times n_phi equally spaced azimuths; weights sum
    to 2 pi.  Used as the converged reference for Bhat(l, m)."""
    x, w = np.polynomial.legendre.leggauss(n_theta)
    z = 0.5 * (x + 1.0)
    wz = 0.5 * w
    ph = 2.0 * math.pi * np.arange(n_phi) / n_phi
    Z, PH = np.meshgrid(z, ph, indexing="ij")
    S = np.sqrt(1.0 - Z * Z)
    dirs = np.stack([(S * np.cos(PH)).ravel(), (S * np.sin(PH)).ravel(), Z.ravel()], axis=1)
    wts = (wz[:, None] * np.full(n_phi, 2.0 * math.pi / n_phi)[None, :]).ravel()
    return dirs, wts
