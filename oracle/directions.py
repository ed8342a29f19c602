"""Hemisphere direction rules for the angular quadrature of the fast spectral
method (Sec. 4.4.1, 3D case).  TEST INFRASTRUCTURE ONLY (see package doc).

The angular integral over e in S^2_+ of the kernel's Fourier factors is even in
e, so any rule on the half sphere whose weights sum to 2*pi (the hemisphere
area) integrates it.  Three rules are provided; each returns (dirs[M,3],
weights[M]) in float64.
"""
import math

import numpy as np


def icosa6():
    """The six axes of the regular icosahedron, weight pi/3 each (an exact
    antipodal 5-design).  Representatives (0,1,g),(0,-1,g),(1,g,0),(-1,g,0),
    (g,0,1),(-g,0,1), g the golden ratio, normalised."""
    g = (1.0 + math.sqrt(5.0)) / 2.0
    raw = np.array([[0.0, 1.0, g], [0.0, -1.0, g], [1.0, g, 0.0],
                    [-1.0, g, 0.0], [g, 0.0, 1.0], [-g, 0.0, 1.0]])
    dirs = raw / math.sqrt(1.0 + g * g)
    return dirs, np.full(6, math.pi / 3.0)


def product(a1: int, a2: int):
    """The (theta_p, phi_q) product grid of the 3D fast method with a1*a2
    points: theta_p = (p + 1/2) pi / a1, phi_q = q pi / a2 (p < a1, q < a2),
    weights proportional to sin(theta_p) and renormalised to sum to 2 pi
    (the area element the printed rule omits)."""
    th = (np.arange(a1) + 0.5) * math.pi / a1
    ph = np.arange(a2) * math.pi / a2
    T, P = np.meshgrid(th, ph, indexing="ij")
    T = T.ravel()
    P = P.ravel()
    dirs = np.stack([np.sin(T) * np.cos(P), np.sin(T) * np.sin(P), np.cos(T)], axis=1)
    w = np.sin(T)
    w = w * (2.0 * math.pi / w.sum())
    return dirs, w


def spiral(m: int):
    """Equal-weight golden-spiral rule on the upper hemisphere: z_p = (p+1/2)/m
    (equal-area bands), azimuth 2 pi p / golden ratio, weight 2 pi / m."""
    p = np.arange(m, dtype=np.float64)
    z = (p + 0.5) / m
    g = (1.0 + math.sqrt(5.0)) / 2.0
    az = 2.0 * math.pi * p / g
    s = np.sqrt(1.0 - z * z)
    dirs = np.stack([s * np.cos(az), s * np.sin(az), z], axis=1)
    return dirs, np.full(m, 2.0 * math.pi / m)


# ---------------------------------------------------------------- spherical designs
# A rule {e_p, w_p} on the half sphere, extended antipodally, integrates every
# polynomial of degree <= t exactly (an antipodal t-design, t odd) iff for every
# even l with 2 <= l <= t - 1 the degree-l zonal sums vanish:
#     r_l = sum_{p,q} w_p w_q P_l(e_p . e_q) / (sum_p w_p)^2 = 0
# (addition theorem: r_l is proportional to sum_m |sum_p w_p Y_lm(e_p)|^2).
# Odd degrees integrate to zero by the antipodal symmetry.

def design_residual(dirs, weights, l: int) -> float:
    """r_l of the rule (>= 0, zero iff degree-l harmonics are integrated exactly)."""
    import scipy.special as sps
    e = np.asarray(dirs, dtype=np.float64)
    w = np.asarray(weights, dtype=np.float64)
    c = np.clip(e @ e.T, -1.0, 1.0)
    return float(w @ sps.eval_legendre(l, c) @ w) / float(w.sum()) ** 2


def design_degree(dirs, weights, tol: float = 1e-12, lmax: int = 80) -> int:
    """Largest odd t such that r_l <= tol for every even l in [2, t-1]."""
    t = 1
    for l in range(2, lmax + 1, 2):
        if design_residual(dirs, weights, l) > tol:
            break
        t = l + 1
    return t


def _sh_even_rows(e, L):
    """Real orthonormal spherical harmonics of the even degrees 2..L at the
    unit vectors e [M, 3], and their gradients in R^3 (the harmonics written
    as Q_l^m(z) Re/Im (x + i y)^m, Q_l^m = P_l^m / (1 - z^2)^{m/2}).
    Returns (Y [R, M], G [R, M, 3])."""
    x, y, z = e[:, 0], e[:, 1], e[:, 2]
    w = x + 1j * y
    Y, G = [], []
    for l in range(2, L + 1, 2):
        for m in range(0, l + 1):
            # Q_m^m = (2m-1)!!, Q_{m+1}^m = (2m+1) z Q_m^m, then the three-term recurrence
            qmm = float(np.prod(np.arange(1, 2 * m, 2))) if m > 0 else 1.0
            qa, da = np.full_like(z, qmm), np.zeros_like(z)
            if l > m:
                qb, db = (2 * m + 1) * z * qmm, np.full_like(z, (2 * m + 1) * qmm)
                for ll in range(m + 2, l + 1):
                    qn = ((2 * ll - 1) * z * qb - (ll + m - 1) * qa) / (ll - m)
                    dn = ((2 * ll - 1) * (qb + z * db) - (ll + m - 1) * da) / (ll - m)
                    qa, da, qb, db = qb, db, qn, dn
                q, dq = qb, db
            else:
                q, dq = qa, da
            nrm = math.sqrt((2 * l + 1) / (4 * math.pi) * math.factorial(l - m) / math.factorial(l + m))
            wm = w ** m
            wm1 = m * w ** (m - 1) if m > 0 else np.zeros_like(w)
            parts = [(nrm, wm.real, wm1.real, -wm1.imag)] if m == 0 else [
                (math.sqrt(2) * nrm, wm.real, wm1.real, -wm1.imag),
                (math.sqrt(2) * nrm, wm.imag, wm1.imag, wm1.real)]
            for c, W, Wx, Wy in parts:
                Y.append(c * q * W)
                G.append(np.stack([c * q * Wx, c * q * Wy, c * dq * W], axis=1))
    return np.array(Y), np.array(G)


def _tangent_frame(e):
    a = np.where(np.abs(e[:, 2:3]) < 0.9, np.array([[0.0, 0.0, 1.0]]), np.array([[1.0, 0.0, 0.0]]))
    t1 = np.cross(e, a)
    t1 /= np.linalg.norm(t1, axis=1, keepdims=True)
    t2 = np.cross(e, t1)
    return t1, t2


def design_terms(m: int) -> int:
    """Even degree L up to which design(m) makes the harmonic sums vanish: the
    largest even L whose conditions sum_{even l = 2..L} (2l + 1) = L (L + 3) / 2
    do not exceed the 2m - 3 free coordinates (2 per point, less a rotation)."""
    L = 0
    while (L + 2) * (L + 5) // 2 <= 2 * m - 3:
        L += 2
    return L


def design(m: int, iters: int = 40):
    """Equal-weight half-sphere rule that is an antipodal spherical design.

    Start: the golden spiral of spiral(m).  Unknowns: two tangent-plane
    coordinates per point.  Equations: sum_p Y_lm(e_p) = 0 for every real
    harmonic of even degree 2 <= l <= L (L from design_terms, fewer equations
    than unknowns).  Iteration (damped minimum-norm Gauss-Newton with a fixed
    damping schedule mu_k = 1e-2 * 0.3^k):
        d = -J^T (J J^T + mu_k I)^{-1} r,   e_p <- normalise(e_p + d_p1 t1 + d_p2 t2),
    stopped when |r| <= 1e-13 sqrt(R); if it stalls, L is lowered by 2 and the
    iteration restarts from the spiral.  Points with z < 0 are then replaced by
    their antipodes.  Returns (dirs [m, 3], weights [m] = 2 pi / m, t) with t
    the degree reached, L + 1."""
    L = design_terms(m)
    while L >= 2:
        e = spiral(m)[0]
        ok = False
        for k in range(iters):
            Y, G = _sh_even_rows(e, L)
            r = Y.sum(axis=1)
            if np.linalg.norm(r) <= 1e-13 * math.sqrt(len(r)):
                ok = True
                break
            t1, t2 = _tangent_frame(e)
            J = np.empty((len(r), 2 * m))
            J[:, 0::2] = np.einsum("rmk,mk->rm", G, t1)
            J[:, 1::2] = np.einsum("rmk,mk->rm", G, t2)
            mu = 1e-2 * 0.3 ** k
            d = -J.T @ np.linalg.solve(J @ J.T + mu * np.eye(len(r)), r)
            e = e + d[0::2, None] * t1 + d[1::2, None] * t2
            e /= np.linalg.norm(e, axis=1, keepdims=True)
        if ok:
            flip = e[:, 2] < 0
            e[flip] = -e[flip]
            return e, np.full(m, 2.0 * math.pi / m), L + 1
        L -= 2
    return spiral(m) + (1,)
