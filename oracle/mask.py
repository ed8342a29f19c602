"""FP64 oracle of the moment-realizability regime mask (Sec. 3.2-3.3, 4.5,
Algorithm 1).  TEST INFRASTRUCTURE ONLY (see package doc).

Per cell (ix, iy) of an nx x ny grid, from the macro fields rho, ux, uy, T and
the per-cell Knudsen number eps:

  * one-cell stencil, clamped at the border (the ghost cells of Sec. 5 copy
    the nearest physical cell): first derivatives by central differences,
    Laplacians by the 5-point formula over dx*dy (Sec. 4.5);
  * xi1 = eps mu / (rho T), xi2 = eps^2 2 kappa^2 / (3 rho^2 T^3) with the
    hard-sphere laws mu = mu0 sqrt(T), kappa = kappa0 sqrt(T) (Sec. 3.1);
  * the 2D-space matrix V_eps1 (a 2x2 block plus h1) and its closed-form
    eigenvalues lambda_a, lambda_b, lambda_c (Sec. 4.5);
  * the ES-BGK -> Boltzmann indicator
      lambda_B = eps^2 (|grad T|^2 / T + |grad u|^2
                        + sqrt((|Lap u|^2 + |Lap rho / rho|^2)(1 + T^2)))
    (Sec. 3.3), |grad u|^2 the Frobenius norm of the 2x2 velocity Jacobian,
    Lap u = Lap ux + Lap uy as the paper writes it (mode 0) or the vector
    norm sqrt(Lap ux^2 + Lap uy^2) (mode 1);
  * Algorithm 1 (regime update) with thresholds eta0, eta1, delta0.

Every value is formed by a fixed sequence of IEEE FP64 operations, each
rounded once (no fused multiply-add), so that an independent implementation
following the same sequence reproduces it bit for bit.

cell_flags: bit 0 SOLID (regime 255, never listed), bit 1 FORCE_BOLTZMANN
(regime 2; the ring of cells around an obstacle forced to the Boltzmann
layer in Sec. 5).  Without an L1 distance the 1 -> 0 switch never fires.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

SOLID = 1
FORCE_BOLTZMANN = 2
REGIME_SOLID = 255


@dataclass
class MaskDesc:
    nx: int
    ny: int
    dx: float
    dy: float
    mu0: float = 1.0
    kappa0: float = 15.0 / 4.0
    eta0: float = 1e-3
    eta1: float = 1e-4
    delta0: float = 1e-4
    laplacian_u_mode: int = 0


def indicators(d: MaskDesc, rho, ux, uy, T, eps):
    """Return (lam_a, lam_b, lam_c, lam_B) arrays [ny][nx] in the canonical
    operation order."""
    nx, ny = d.nx, d.ny
    ix = np.arange(nx)
    iy = np.arange(ny)
    iL = np.maximum(ix - 1, 0)
    iR = np.minimum(ix + 1, nx - 1)
    jL = np.maximum(iy - 1, 0)
    jR = np.minimum(iy + 1, ny - 1)
    two_dx = 2.0 * d.dx
    two_dy = 2.0 * d.dy
    dxdy = d.dx * d.dy

    def ddx(q):
        return (q[:, iR] - q[:, iL]) / two_dx

    def ddy(q):
        return (q[jR, :] - q[jL, :]) / two_dy

    def lap(q):
        return ((((q[:, iL] + q[:, iR]) + q[jL, :]) + q[jR, :]) - 4.0 * q) / dxdy

    uxx = ddx(ux)
    uxy = ddy(ux)
    uyx = ddx(uy)
    uyy = ddy(uy)
    Tx = ddx(T)
    Ty = ddy(T)
    sqT = np.sqrt(T)
    mu = d.mu0 * sqT
    kap = d.kappa0 * sqT
    xi1 = (eps * mu) / (rho * T)
    xi2 = ((eps * eps) * (2.0 * (kap * kap))) / (((((3.0 * rho) * rho) * T) * T) * T)
    c43 = 4.0 / 3.0
    c23 = 2.0 / 3.0
    a1 = c43 * uxx - c23 * uyy
    a2 = Tx * Tx
    b1 = uxy + uyx
    b2 = Tx * Ty
    c1 = c43 * uyy - c23 * uxx
    c2 = Ty * Ty
    h1 = (-c23) * (uxx + uyy)
    dd = xi1 * b1 + xi2 * b2
    p = xi1 * (a1 - c1) + xi2 * (a2 - c2)
    sq = np.sqrt(p * p + 4.0 * (dd * dd))
    s = (((a1 * xi1) + (a2 * xi2)) + (c1 * xi1)) + (c2 * xi2)
    lam_a = 0.5 * ((sq - s) + 2.0)
    lam_b = 0.5 * (((-sq) - s) + 2.0)
    lam_c = 1.0 - xi1 * h1
    gT2 = Tx * Tx + Ty * Ty
    gu2 = ((uxx * uxx + uxy * uxy) + uyx * uyx) + uyy * uyy
    lux = lap(ux)
    luy = lap(uy)
    lr = lap(rho) / rho
    if d.laplacian_u_mode == 0:
        lu = lux + luy
        lu2 = lu * lu
    else:
        lu2 = lux * lux + luy * luy
    inner = (lu2 + lr * lr) * (1.0 + T * T)
    lam_B = (eps * eps) * ((gT2 / T + gu2) + np.sqrt(inner))
    return lam_a, lam_b, lam_c, lam_B


def regime_update(d: MaskDesc, lam, regime_in, l1dist=None, flags=None, valid=None):
    """Algorithm 1 applied cell by cell (vectorised).  Cells marked invalid
    (non-positive density or temperature, negative eps, non-finite values)
    keep their regime; regime codes other than 0, 1, 2 and 255 are kept too."""
    lam_a, lam_b, lam_c, lam_B = lam
    r = np.asarray(regime_in)
    big_B = np.abs(lam_B) > d.eta1
    near_one = (np.abs(lam_a - 1.0) <= d.eta0) & (np.abs(lam_b - 1.0) <= d.eta0) & \
        (np.abs(lam_c - 1.0) <= d.eta0)
    if l1dist is None:
        close = np.zeros(r.shape, dtype=bool)
    else:
        close = np.asarray(l1dist) <= d.delta0
    out = r.astype(np.uint8).copy()
    # regime 2: stay iff lambda_B > eta1, else fall back to ES-BGK
    out[r == 2] = np.where(big_B, 2, 1)[r == 2]
    # regime 1: up to 2 on lambda_B; down to 0 only if V_eps1 ~ I and f ~ M
    r1 = np.where(big_B, 2, np.where(near_one & close, 0, 1))
    out[r == 1] = r1[r == 1]
    # regime 0: up to 1 when V_eps1 leaves the identity; never to 2 directly
    out[r == 0] = np.where(near_one, 0, 1)[r == 0]
    out[r == REGIME_SOLID] = REGIME_SOLID
    if valid is not None:
        out[~valid] = r[~valid]
    if flags is not None:
        fl = np.asarray(flags)
        out[(fl & FORCE_BOLTZMANN) != 0] = 2
        out[(fl & SOLID) != 0] = REGIME_SOLID
    return out


def input_valid(rho, ux, uy, T, eps, lam):
    """rho > 0, T > 0, eps >= 0 and every input and indicator finite."""
    with np.errstate(invalid="ignore"):
        ok = (rho > 0) & (T > 0) & (eps >= 0)
    for x in (rho, ux, uy, T, eps) + tuple(lam):
        ok &= np.isfinite(x)
    return ok


def realizability_mask(d: MaskDesc, rho, ux, uy, T, eps, regime_in, l1dist=None, flags=None):
    """Return (regime_out [ny][nx] uint8, ascending int32 list of regime-2
    linear indices iy*nx + ix, diag [ny*nx][4] = (lam_a, lam_b, lam_c, lam_B))."""
    lam = indicators(d, rho, ux, uy, T, eps)
    valid = input_valid(rho, ux, uy, T, eps, lam)
    out = regime_update(d, lam, regime_in, l1dist, flags, valid)
    idx = np.flatnonzero(out.ravel() == 2).astype(np.int32)
    diag = np.stack([x.ravel() for x in lam], axis=1)
    return out, idx, diag, int((~valid).sum())


def margin_cells(d: MaskDesc, lam, rel: float = 1e-12) -> int:
    """Cells whose decision quantities sit within ``rel`` of a threshold."""
    lam_a, lam_b, lam_c, lam_B = lam
    cnt = np.abs(np.abs(lam_B) - d.eta1) <= rel * d.eta1
    for x in (lam_a, lam_b, lam_c):
        cnt |= np.abs(np.abs(x - 1.0) - d.eta0) <= rel * d.eta0
    return int(cnt.sum())
