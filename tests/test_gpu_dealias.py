"""Dealiased (3/2-rule) plans against the oracle's truncated convolution
without wrap-around (through the C ABI)."""
import numpy as np
import pytest

import bz_inputs as gen
from oracle import spectral
from tests.gpu_util import lib_kwargs, oracle_plan

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


@pytest.mark.parametrize("n,rule,m,prec", [(16, "icosa6", 6, "fp64"), (16, "icosa6", 6, "fp32"),
                                           (32, "spiral", 32, "fp32"), (32, "spiral", 32, "fp64")])
def test_dealiased_against_oracle(n, rule, m, prec):
    import paper_2505_03360_amd as bz
    print("case dealias", n, rule, m, prec, flush=True)
    L = 8.0
    f = gen.shock_batch(3, n, L, seed=70 + n)
    rows = [2, 0]
    plan = oracle_plan(n, rule=rule, m=m)
    ref = [spectral.project(spectral.collide_dealiased(f[r], plan, op=spectral.collide_fft), n, L) for r in rows]
    loss = [spectral.collide_parts(f[r], plan)[2] for r in rows]
    col = bz.Collider(n, len(rows), L=L, precision=bz.BZ_FP32 if prec == "fp32" else bz.BZ_FP64, dealias=1,
                      **lib_kwargs(rule, m))
    idx = torch.tensor(rows, dtype=torch.int32, device="cuda")
    q = col(torch.from_numpy(f).cuda(), idx=idx).cpu().numpy()
    tol = 1e-5 if prec == "fp32" else 1e-12
    for c in range(len(rows)):
        err = spectral.rel_err(q[c], ref[c], loss[c])
        print(f"  cell {c}: err {err:.3e}", flush=True)
        assert err <= tol
    if prec == "fp64":
        # the result is the dealiased operator, not the circular one (their
        # difference on these cells, ~1e-4 of ||Q||, is below FP32 rounding of
        # the gain and loss terms, so this is checked in FP64)
        circ = spectral.project(spectral.collide(f[rows[0]], plan), n, L)
        assert np.linalg.norm(ref[0] - circ) > 1e3 * np.linalg.norm(q[0] - ref[0])
    col.close()


def test_benchmarked_dealiased_batch_sampled():
    """The benchmarked dealiased launch (256 shock cells, N = 32, M = 32 spiral,
    FP32 + FP64 projection, padded 48^3 sub-plan): sampled cells against the
    oracle's truncated convolution; identical inputs give identical outputs."""
    import paper_2505_03360_amd as bz
    print("case dealias 256 cells", flush=True)
    n, L, cells = 32, 8.0, 256
    f = gen.shock_batch(cells, n, L, seed=2)
    f[200] = f[3]
    col = bz.Collider(n, cells, L=L, m=32, dir_kind=bz.BZ_DIRS_SPIRAL, precision=bz.BZ_FP32, dealias=1)
    q = col(torch.from_numpy(f).cuda())
    torch.cuda.synchronize()
    q = q.cpu().numpy()
    plan = oracle_plan(n, rule="spiral", m=32)
    for c in (0, 131, 255):
        ref = spectral.project(spectral.collide_dealiased(f[c], plan, op=spectral.collide_fft), n, L)
        loss = spectral.collide_fft(f[c], plan, parts=True)[2]
        err = spectral.rel_err(q[c], ref, loss)
        print(f"  cell {c}: err {err:.3e}", flush=True)
        assert err <= 1e-5
    assert np.array_equal(q[200], q[3])
    col.close()
