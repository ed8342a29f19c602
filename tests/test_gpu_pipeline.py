"""Kinetic cells feed the regime mask from their own distributions: moments
and L1 distance from resident f (bz_cell_moments) -> realizability mask with
the L1 criterion (bz_realizability_mask), so that cells near equilibrium
switch from the kinetic layer 1 to the fluid layer 0 (Algorithm 1)."""
import math

import numpy as np
import pytest

from oracle import kinetic, mask

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def test_moments_feed_the_mask():
    import paper_2505_03360_amd as bz
    print("case moments -> mask", flush=True)
    nx = ny = 24
    n, L = 16, 8.0
    rng = np.random.default_rng(12)
    X, Y = np.meshgrid(np.arange(nx) / nx, np.arange(ny) / ny, indexing="xy")
    rho = 1.0 + 0.05 * np.sin(2 * math.pi * X) * np.cos(2 * math.pi * Y)
    T = 1.0 + 0.05 * np.cos(2 * math.pi * X)
    ux = 0.1 * np.sin(2 * math.pi * Y)
    uy = 0.05 * np.cos(2 * math.pi * X)
    v = (np.arange(n) - n // 2) * (2 * L / n)
    V1, V2, V3 = np.meshgrid(v, v, v, indexing="ij")
    f = np.empty((ny * nx, n, n, n))
    for iy in range(ny):
        for ix in range(nx):
            c = iy * nx + ix
            u = [ux[iy, ix], uy[iy, ix], 0.0]
            M = kinetic.maxwellian(rho[iy, ix], u, T[iy, ix], n, L)
            a = 0.05 if ix >= nx // 2 else 0.0  # a shear-stress departure in the right half
            f[c] = M * (1.0 + a * (V1 - u[0]) * (V2 - u[1]) / T[iy, ix]) * (1.0 + 1e-3 * rng.uniform(-1, 1))
    ft = torch.from_numpy(f).cuda()
    mom = bz.cell_moments(ft, L)
    torch.cuda.synchronize()
    for c in (0, nx // 2 + 3, ny * nx - 1):  # spot checks against the oracle
        r_, u_, T_ = kinetic.moments(f[c], n, L)
        assert abs(float(mom["rho"][c]) - r_) <= 1e-13 * r_ and abs(float(mom["T"][c]) - T_) <= 1e-12 * T_
        assert abs(float(mom["l1"][c]) - kinetic.l1_distance(f[c], n, L)) <= 1e-12 * r_
    grid = {k: t.view(ny, nx).contiguous() for k, t in mom.items()}
    eps = torch.full((ny, nx), 1e-4, dtype=torch.float64, device="cuda")
    regime_in = torch.ones((ny, nx), dtype=torch.uint8, device="cuda")
    desc = bz.mask_desc(nx, ny, 1.0 / nx, 1.0 / ny, eta0=1e-3, eta1=1e3, delta0=1e-3)
    rout, idx, counts, _ = bz.realizability_mask(desc, grid["rho"], grid["u1"], grid["u2"], grid["T"], eps,
                                                 regime_in, l1dist=grid["l1"])
    torch.cuda.synchronize()
    h = {k: t.cpu().numpy() for k, t in grid.items()}
    d = mask.MaskDesc(nx, ny, 1.0 / nx, 1.0 / ny, eta0=1e-3, eta1=1e3, delta0=1e-3)
    lam = mask.indicators(d, h["rho"], h["u1"], h["u2"], h["T"], eps.cpu().numpy())
    assert mask.margin_cells(d, lam) == 0
    ref, ref_idx, _, nbad = mask.realizability_mask(d, h["rho"], h["u1"], h["u2"], h["T"], eps.cpu().numpy(),
                                                    regime_in.cpu().numpy(), l1dist=h["l1"])
    out = rout.cpu().numpy()
    assert np.array_equal(out, ref)
    assert nbad == 0 and int(counts[1]) == 0
    # the equilibrium half switches to the fluid layer, the sheared half stays kinetic
    assert (out[:, : nx // 2] == 0).all() and (out[:, nx // 2:] == 1).all()
