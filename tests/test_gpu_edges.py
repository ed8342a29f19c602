"""Edge cases of the newer entry points on the GPU: a device-side cell count
(ncells_dev, as in graph capture) smaller than the launch capacity, a zero
device count, and empty batches; rows beyond the live count are untouched."""
import numpy as np
import pytest

import bz_inputs as gen
from oracle import kinetic, spectral

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def dev_count(k):
    return torch.tensor([k], dtype=torch.int32, device="cuda")


def test_moments_device_count():
    import paper_2505_03360_amd as bz
    print("case edges moments", flush=True)
    n, L = 16, 8.0
    f = gen.shock_batch(5, n, L, seed=31)
    ft = torch.from_numpy(f).cuda()
    out = {k: torch.full((5,), -7.0, dtype=torch.float64, device="cuda") for k in ("rho", "u1", "u2", "u3", "T", "l1")}
    bz.cell_moments(ft, L, ncells=5, ncells_dev=dev_count(3), out=out)
    rho = out["rho"].cpu().numpy()
    for c in range(3):
        assert abs(rho[c] - kinetic.moments(f[c], n, L)[0]) <= 1e-13 * rho[c]
    assert (rho[3:] == -7.0).all()
    bz.cell_moments(ft, L, ncells=5, ncells_dev=dev_count(0), out=out)  # nothing written
    torch.cuda.synchronize()
    assert (out["rho"].cpu().numpy()[3:] == -7.0).all()


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_imex_and_dealias_device_count(prec):
    import paper_2505_03360_amd as bz
    print("case edges imex/dealias", prec, flush=True)
    n, L = 16, 8.0
    p = bz.BZ_FP32 if prec == "fp32" else bz.BZ_FP64
    f = torch.from_numpy(gen.shock_batch(4, n, L, seed=32)).cuda()
    tr = torch.zeros_like(f)
    for dealias in (0, 1):
        col = bz.Collider(n, 4, L=L, m=6, dir_kind=bz.BZ_DIRS_ICOSA6, precision=p, dealias=dealias)
        full = col(f)
        part = torch.full_like(full, -3.0)
        col(f, ncells=4, ncells_dev=dev_count(2), out=part)
        torch.cuda.synchronize()
        assert torch.equal(part[:2], full[:2]) and bool((part[2:] == -3.0).all())
        if not dealias:
            o = torch.full_like(f, -5.0)
            col.imex_euler(f, tr, 0.01, eps=0.1, ncells=4, ncells_dev=dev_count(1), out=o)
            ref = col.imex_euler(f, tr, 0.01, eps=0.1)
            torch.cuda.synchronize()
            assert torch.equal(o[:1], ref[:1]) and bool((o[1:] == -5.0).all())
        col.close()


def test_esbgk_device_count_and_empty():
    import paper_2505_03360_amd as bz
    print("case edges esbgk", flush=True)
    n, L = 16, 8.0
    f = torch.from_numpy(gen.shock_batch(3, n, L, seed=33)).cuda()
    full = bz.esbgk_collide(f, L)
    part = torch.full_like(full, 2.0)
    bz.esbgk_collide(f, L, ncells=3, ncells_dev=dev_count(2), out=part)
    torch.cuda.synchronize()
    assert torch.equal(part[:2], full[:2]) and bool((part[2:] == 2.0).all())
    # empty batches return at once
    bz.bz_esbgk_collide(bz.BzEsbgkDesc(n, L, -0.5, 1.0), 0, 0, 0, 0, 0)
    bz.bz_cell_moments(n, L, 0, bz.BZ_FP64, 0, 0, 0, bz.BzMomentsOut())
