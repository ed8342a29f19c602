"""Precision sweep against the oracle: N in {32, 48}, M in {32, 64},
gamma in {0, 0.5, 1}, FP32 (fused kernel at N=32, plain passes at N=48) and
FP64, on two shock cells each; moments conserved after projection."""
import numpy as np
import pytest

import bz_inputs as gen
from oracle import spectral
from tests.gpu_util import cell_errors, oracle_cells, oracle_plan

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


@pytest.mark.parametrize("n", [32, 48])
@pytest.mark.parametrize("m", [32, 64])
@pytest.mark.parametrize("gamma", [0.0, 0.5, 1.0])
def test_sweep_against_oracle(n, m, gamma):
    import paper_2505_03360_amd as bz
    print("case sweep", n, m, gamma, flush=True)
    f = gen.shock_batch(2, n, 8.0, seed=4)
    ref, loss = oracle_cells(f, oracle_plan(n, m=m, gamma=gamma))
    ft = torch.from_numpy(f).cuda()
    for prec, tol in ((bz.BZ_FP32, 1e-5), (bz.BZ_FP64, 1e-12)):
        col = bz.Collider(n, 2, L=8.0, m=m, dir_kind=bz.BZ_DIRS_SPIRAL, gamma=gamma, precision=prec)
        q = col(ft)
        torch.cuda.synchronize()
        q = q.cpu().numpy()
        err = cell_errors(q, ref, loss)
        print(f"  n={n} m={m} gamma={gamma} prec={'fp32' if prec else 'fp64'} max err {err.max():.3e}", flush=True)
        assert err.max() <= tol, err
        assert max(spectral.moment_drift(q[c], n, 8.0) for c in range(2)) <= 1e-12
