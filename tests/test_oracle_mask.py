"""Pins of the regime-mask oracle (Sec. 3.2-3.3, 4.5, Algorithm 1).

  P11  closed-form eigenvalues vs numpy.linalg.eigvalsh of V_eps1 assembled
       from its definition I - eps mu/(rho T) D(u) - eps^2 (2/3)
       kappa^2/(rho^2 T^3) grad T (x) grad T, with derivatives taken by
       numpy.gradient (interior cells)
  P12  Algorithm 1 branch table on hand-built fields whose indicators are
       known exactly (uniform state, pure shear, flags)
"""
import json
import math
import os

import numpy as np
import pytest

import bz_inputs as gen
from oracle import mask as om
from oracle import spectral

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def desc(nx, ny, **kw):
    return om.MaskDesc(nx=nx, ny=ny, dx=1.0 / nx, dy=1.0 / ny, **kw)


def test_p11_eigenvalues_against_eigvalsh():
    nx = ny = 24
    rho, ux, uy, T = gen.random_macro_field(nx, ny, seed=5)
    d = desc(nx, ny)
    eps = np.full((ny, nx), 3e-3)
    la, lb, lc, lB = om.indicators(d, rho, ux, uy, T, eps)
    # independent assembly of V_eps1 from its definition
    dux_dy, dux_dx = np.gradient(ux, d.dy, d.dx)
    duy_dy, duy_dx = np.gradient(uy, d.dy, d.dx)
    dT_dy, dT_dx = np.gradient(T, d.dy, d.dx)
    for iy in range(1, ny - 1):
        for ix in range(1, nx - 1):
            J = np.zeros((3, 3))  # J[a, b] = d u_a / d x_b, u_z = 0, d/dz = 0
            J[0, 0], J[0, 1] = dux_dx[iy, ix], dux_dy[iy, ix]
            J[1, 0], J[1, 1] = duy_dx[iy, ix], duy_dy[iy, ix]
            D = J + J.T - (2.0 / 3.0) * np.trace(J) * np.eye(3)
            g = np.array([dT_dx[iy, ix], dT_dy[iy, ix], 0.0])
            r, t, e = rho[iy, ix], T[iy, ix], eps[iy, ix]
            mu, kap = d.mu0 * math.sqrt(t), d.kappa0 * math.sqrt(t)
            V = np.eye(3) - e * mu / (r * t) * D - e * e * (2.0 / 3.0) * kap ** 2 / (r * r * t ** 3) * np.outer(g, g)
            ev = np.sort(np.linalg.eigvalsh(V))
            mine = np.sort([la[iy, ix], lb[iy, ix], lc[iy, ix]])
            assert np.abs(ev - mine).max() <= 1e-14 * 4, (iy, ix, ev, mine)


def test_lambda_b_independent_interior():
    nx = ny = 20
    rho, ux, uy, T = gen.random_macro_field(nx, ny, seed=9)
    d = desc(nx, ny, laplacian_u_mode=1)
    eps = np.full((ny, nx), 1e-2)
    lB = om.indicators(d, rho, ux, uy, T, eps)[3]
    s = (slice(1, -1), slice(1, -1))

    def lap(q):
        return (q[1:-1, :-2] + q[1:-1, 2:] + q[:-2, 1:-1] + q[2:, 1:-1] - 4 * q[1:-1, 1:-1]) / (d.dx * d.dy)
    gy, gx = np.gradient(T, d.dy, d.dx)
    Ju = [np.gradient(q, d.dy, d.dx) for q in (ux, uy)]
    gu2 = sum(a[s] ** 2 + b[s] ** 2 for a, b in Ju)
    lu2 = lap(ux) ** 2 + lap(uy) ** 2
    ref = eps[s] ** 2 * ((gx[s] ** 2 + gy[s] ** 2) / T[s] + gu2 +
                         np.sqrt((lu2 + (lap(rho) / rho[s]) ** 2) * (1 + T[s] ** 2)))
    assert np.abs(lB[s] - ref).max() <= 1e-12 * np.abs(ref).max()


def test_p12_uniform_state_branches():
    nx, ny = 6, 5
    d = desc(nx, ny, eta0=1e-3, eta1=1e-4, delta0=1e-3)
    one = np.ones((ny, nx))
    regime = np.array([0, 1, 2, 1, 2, 0] * ny, dtype=np.uint8).reshape(ny, nx)
    lam = om.indicators(d, one, 0 * one, 0 * one, one, 1e-2 * one)
    assert all(np.all(x == 1.0) for x in lam[:3]) and np.all(lam[3] == 0.0)
    out = om.regime_update(d, lam, regime)
    # Euler stays Euler; ES-BGK without an L1 distance stays; Boltzmann drops to 1
    exp = np.array([0, 1, 1, 1, 1, 0] * ny, dtype=np.uint8).reshape(ny, nx)
    assert np.array_equal(out, exp)
    l1 = np.full((ny, nx), 5e-4)
    l1[:, 3] = 2e-3
    out = om.regime_update(d, lam, regime, l1dist=l1)
    exp = np.array([0, 0, 1, 1, 1, 0] * ny, dtype=np.uint8).reshape(ny, nx)
    assert np.array_equal(out, exp)
    flags = np.zeros((ny, nx), dtype=np.uint8)
    flags[0, 0] = om.FORCE_BOLTZMANN
    flags[1, 1] = om.SOLID
    flags[2, 2] = om.SOLID | om.FORCE_BOLTZMANN
    out = om.regime_update(d, lam, regime, flags=flags)
    assert out[0, 0] == 2 and out[1, 1] == 255 and out[2, 2] == 255
    o2, idx, diag, nbad = om.realizability_mask(d, one, 0 * one, 0 * one, one, 1e-2 * one, regime, flags=flags)
    assert list(idx) == [0]


def test_p12_shear_branches():
    """ux = g y: interior cells have b1 = g and zero Laplacians, so
    lambda_{a,b} = 1 -+ xi1 |g|, lambda_c = 1, lambda_B = eps^2 g^2."""
    nx, ny = 7, 9
    dx = dy = 0.125
    g = 0.5
    Y = np.repeat((np.arange(ny) * dy)[:, None], nx, axis=1)
    ux = g * Y
    one = np.ones((ny, nx))
    eps = 1e-2
    d = om.MaskDesc(nx=nx, ny=ny, dx=dx, dy=dy, mu0=1.0, kappa0=15 / 4,
                    eta0=0.5 * eps * g, eta1=0.5 * eps * eps * g * g)
    la, lb, lc, lB = om.indicators(d, one, ux, 0 * one, one, eps * one)
    inner = (slice(1, -1), slice(None))
    xi1 = eps  # rho = T = 1, mu0 = 1
    assert np.allclose(la[inner], 1 + xi1 * g, rtol=0, atol=1e-15)
    assert np.allclose(lb[inner], 1 - xi1 * g, rtol=0, atol=1e-15)
    assert np.all(lc == 1.0)
    assert np.allclose(lB[inner], eps * eps * g * g, rtol=1e-12)
    for rin, expect in [(0, 1), (1, 2), (2, 2)]:
        out = om.regime_update(d, (la, lb, lc, lB), np.full((ny, nx), rin, np.uint8))
        assert np.all(out[inner] == expect), (rin, out)


def test_paper_parameter_fixture():
    with open(os.path.join(GOLDEN, "paper_parameters.json")) as fh:
        p = json.load(fh)
    assert round(spectral.default_R(p["velocity_box_L"]), 1) == p["R_printed_approx"]
    from oracle import directions
    d, w = directions.product(p["A1"], p["A2"])
    assert len(w) == p["A1"] * p["A2"]
    t1 = p["tests"]["test1_sod"]
    assert t1["eta1"] < t1["eta0"]


def test_compaction_ascending_and_margin():
    nx = ny = 32
    rho, ux, uy, T = gen.random_macro_field(nx, ny, seed=2)
    d = desc(nx, ny)
    eps = np.full((ny, nx), 1e-3)
    lam = om.indicators(d, rho, ux, uy, T, eps)
    d.eta1 = float(np.quantile(lam[3], 0.8))
    d.eta1 *= 1.0 + 1e-9
    regime = np.ones((ny, nx), np.uint8)
    out, idx, diag, nbad = om.realizability_mask(d, rho, ux, uy, T, eps, regime)
    assert np.all(np.diff(idx) > 0)
    assert len(idx) == int((out == 2).sum())
    assert om.margin_cells(d, lam) == 0


# ---------------------------------------------------------------- border (ghost cells)
# At the border the stencil reads the nearest cell in place of the missing
# neighbour (the ghost cells of Sec. 5 copy it).  For fields linear or
# quadratic in x or y this gives closed forms that differ from the interior:
#   first derivative of a x at ix = 0 and nx-1:  a dx / (2 dx) = a / 2;
#   Laplacian of b x^2 (x = ix dx) over dx dy:
#     ix = 0:      (q1 - q0) / (dx dy)             =  b dx / dy,
#     ix = nx-1:   (q[nx-2] - q[nx-1]) / (dx dy)   = -b (2 nx - 3) dx / dy,
#     interior:    2 b dx / dy.
def test_border_first_derivative_of_linear_temperature():
    """T = 1 + a x, rho = 1, u = 0: lambda_a = lambda_c = 1,
    lambda_b = 1 - xi2 Tx^2, lambda_B = eps^2 Tx^2 / T with Tx = a/2 on the
    first and last columns and a inside; likewise along y."""
    nx, ny = 9, 7
    dx, dy = 0.1, 0.2
    a, eps = 0.3, 1e-2
    for axis in ("x", "y"):
        X = np.arange(nx)[None, :] * dx + 0 * np.arange(ny)[:, None]
        Y = np.arange(ny)[:, None] * dy + 0 * np.arange(nx)[None, :]
        T = 1.0 + a * (X if axis == "x" else Y)
        one = np.ones((ny, nx))
        d = om.MaskDesc(nx=nx, ny=ny, dx=dx, dy=dy)
        la, lb, lc, lB = om.indicators(d, one, 0 * one, 0 * one, T, eps * one)
        idx = np.arange(nx if axis == "x" else ny)
        border = (idx == 0) | (idx == idx[-1])
        g = np.where(border, a / 2, a)
        G = np.broadcast_to(g[None, :] if axis == "x" else g[:, None], (ny, nx))
        kap = d.kappa0 * np.sqrt(T)
        xi2 = eps * eps * 2 * kap * kap / (3 * T ** 3)
        assert np.allclose(lB, eps * eps * G * G / T, rtol=1e-13, atol=0)
        assert np.allclose(lb, 1 - xi2 * G * G, rtol=0, atol=1e-15)
        assert np.all(la == 1.0) and np.all(lc == 1.0)


def test_border_laplacian_of_quadratic_density():
    """rho = 1 + b x^2, T = 1, u = 0: lambda_B = eps^2 sqrt(2) |Lap rho| / rho
    with the one-sided border Laplacians above (and the same along y)."""
    nx, ny = 8, 6
    dx, dy = 0.125, 0.25
    b, eps = 0.7, 1e-2
    for axis in ("x", "y"):
        nn, h, hh = (nx, dx, dy) if axis == "x" else (ny, dy, dx)
        i = np.arange(nn)
        lap = np.full(nn, 2 * b * h / hh)
        lap[0] = b * h / hh
        lap[-1] = -b * (2 * nn - 3) * h / hh
        r1 = 1.0 + b * (i * h) ** 2
        if axis == "x":
            rho = np.broadcast_to(r1[None, :], (ny, nx)).copy()
            LAP = np.broadcast_to(lap[None, :], (ny, nx))
        else:
            rho = np.broadcast_to(r1[:, None], (ny, nx)).copy()
            LAP = np.broadcast_to(lap[:, None], (ny, nx))
        one = np.ones((ny, nx))
        d = om.MaskDesc(nx=nx, ny=ny, dx=dx, dy=dy)
        lB = om.indicators(d, rho, 0 * one, 0 * one, one, eps * one)[3]
        assert np.allclose(lB, eps * eps * math.sqrt(2) * np.abs(LAP) / rho, rtol=1e-13, atol=0)


def test_border_shear_rows():
    """ux = g y: the first and last rows see d ux/dy = g/2, so
    lambda_{a,b} = 1 -+ xi1 g/2 and lambda_B = eps^2 (g/2)^2 there, plus the
    one-sided Laplacian of ux: (q1 - q0)/(dx dy) = g dy/(dx dy) = g/dx on the
    first row and -g/dx on the last (scalar mode: Lap u = Lap ux)."""
    nx, ny = 5, 8
    dx = dy = 0.125
    g, eps = 0.5, 1e-2
    Y = np.repeat((np.arange(ny) * dy)[:, None], nx, axis=1)
    one = np.ones((ny, nx))
    d = om.MaskDesc(nx=nx, ny=ny, dx=dx, dy=dy)
    la, lb, lc, lB = om.indicators(d, one, g * Y, 0 * one, one, eps * one)
    for row in (0, ny - 1):
        assert np.allclose(la[row], 1 + eps * g / 2, rtol=0, atol=1e-15)
        assert np.allclose(lb[row], 1 - eps * g / 2, rtol=0, atol=1e-15)
        lap = g / dx
        assert np.allclose(lB[row], eps * eps * ((g / 2) ** 2 + math.sqrt(2) * lap), rtol=1e-13, atol=0)
