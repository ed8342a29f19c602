"""GPU parity of bz_collide_batch against the FP64 oracle, through the C ABI.

Tolerance (per cell): ||Q_gpu - Q_ref||_2 / max(||Q_ref||_2, 0.05 ||loss_ref||_2)
<= 1e-12 for the FP64 path and <= 1e-5 for the FP32 path (FP32 transforms,
multipliers, products and accumulation; FP64 projection).  The floor keeps
near-equilibrium cells, where Q is a small difference of gain and loss, from
dividing by ~0.  Conservation after projection: max_i |C_i Q| / sum |C_ij Q_j|
<= 1e-12.
"""
import numpy as np
import pytest

import bz_inputs as gen
from oracle import spectral
from tests.gpu_util import cell_errors, lib_kwargs, oracle_cells, oracle_plan

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def collider(n, cells, precision, rule="spiral", m=32, **kw):
    import paper_2505_03360_amd as bz
    args = dict(L=8.0, precision=precision)
    args.update(lib_kwargs(rule, m))
    args.update(kw)
    return bz.Collider(n, cells, **args)


def run(col, f_np, f_dtype=torch.float64, idx=None, scatter=False, ncells_dev=None, out=None):
    f = torch.from_numpy(f_np).to("cuda", f_dtype).contiguous()
    ii = None if idx is None else torch.as_tensor(idx, dtype=torch.int32, device="cuda")
    q = col(f, idx=ii, scatter=scatter, ncells_dev=ncells_dev, out=out)
    torch.cuda.synchronize()
    return q.cpu().numpy()


def label(*a):
    print("case", *a, flush=True)


@pytest.mark.parametrize("precision,tol", [(0, 1e-12), (1, 1e-5)])
def test_single_cell_n16_icosa6(precision, tol):
    """One cell, N=16 on [-8,8]^3, six icosahedral directions, hard spheres,
    a seeded mix of two Maxwellians."""
    import paper_2505_03360_amd as bz
    label("n16 icosa6", precision)
    f = gen.bimaxwellian_batch(1, 16, 8.0, seed=1)
    col = collider(16, 1, precision, rule="icosa6", m=6)
    q = run(col, f)
    ref, loss = oracle_cells(f, oracle_plan(16, rule="icosa6", m=6))
    err = cell_errors(q, ref, loss)
    assert err.max() <= tol, err
    assert spectral.moment_drift(q[0], 16, 8.0) <= 1e-12
    if precision == bz.BZ_FP32:
        assert col.transform == bz.BZ_XF_FUSED


@pytest.mark.parametrize("precision,tol,transform", [(0, 1e-12, 2), (1, 1e-5, 1), (1, 1e-5, 2)])
def test_ragged_gather_scatter_n16(precision, tol, transform):
    """37 cells (a ragged count) gathered from 100 resident rows by an index
    list, written back by scatter; untouched rows keep their sentinel."""
    label("n16 ragged", precision, transform)
    n = 16
    allf = gen.bimaxwellian_batch(100, n, 8.0, seed=21)
    rng = np.random.default_rng(5)
    idx = np.sort(rng.choice(100, size=37, replace=False)).astype(np.int32)
    col = collider(n, 40, precision, rule="spiral", m=8, transform=transform)
    out = torch.full((100, n, n, n), 7.0, dtype=torch.float64, device="cuda")
    q = run(col, allf, idx=idx, scatter=True, out=out)
    ref, loss = oracle_cells(allf[idx], oracle_plan(n, rule="spiral", m=8))
    err = cell_errors(q[idx], ref, loss)
    assert err.max() <= tol, err
    rest = np.setdiff1d(np.arange(100), idx)
    assert np.all(q[rest] == 7.0)


@pytest.mark.parametrize("precision,tol,cells", [(0, 1e-12, 3), (1, 1e-5, 6)])
def test_n32_m32_shock_cells(precision, tol, cells):
    """N=32, M=32 golden-spiral directions, Mott-Smith shock mixtures."""
    label("n32 m32", precision)
    f = gen.shock_batch(cells, 32, 8.0, seed=2)
    col = collider(32, cells, precision)
    q = run(col, f)
    ref, loss = oracle_cells(f, oracle_plan(32))
    err = cell_errors(q, ref, loss)
    print("max err", err.max(), flush=True)
    assert err.max() <= tol, err
    for c in range(cells):
        assert spectral.moment_drift(q[c], 32, 8.0) <= 1e-12


def test_n32_full_batch_sampled():
    """The benchmarked launch: 256 shock cells, N=32, M=32 spherical design
    (degree 9), FP32 fused + FP64 projection.  Every cell is checked against
    the FP64 GPU path of the same launch size (itself checked against the
    oracle to 1e-12 on sampled cells, below and in the next test) with the
    near-equilibrium floor of the oracle's loss term; eight cells directly
    against the oracle; every cell for conservation and finiteness."""
    import paper_2505_03360_amd as bz
    from tests.gpu_util import floored_errors, oracle_loss_norms, oracle_plan_of
    label("n32 full batch")
    f = gen.shock_batch(256, 32, 8.0, seed=2)
    col = collider(32, 256, 1, rule="design")
    assert col.transform == bz.BZ_XF_FUSED
    q = run(col, f, f_dtype=torch.float64)
    assert np.isfinite(q).all()
    col64 = collider(32, 256, 0, rule="design")
    q64 = run(col64, f, f_dtype=torch.float64)
    oplan = oracle_plan_of(col.plan, 32, 32)
    sample = [0, 31, 77, 128, 160, 200, 233, 255]
    ref, loss = oracle_cells(f[sample], oplan)
    err = cell_errors(q[sample], ref, loss)
    assert err.max() <= 1e-5, err
    assert cell_errors(q64[sample], ref, loss).max() <= 1e-12
    errs, n_cancel = floored_errors(q, q64, oracle_loss_norms(f, oplan))
    print("all cells: max", errs.max(), "median", np.median(errs), "cancellation-dominated", n_cancel, flush=True)
    assert errs.max() <= 1e-5, (errs.argmax(), errs.max())
    drift = max(spectral.moment_drift(q[c], 32, 8.0) for c in range(0, 256, 15))
    assert drift <= 1e-12


def test_n32_fp64_full_batch_sampled():
    """The FP64 GPU path the FP32 speedup is measured against, in its benchmarked
    launch (256 cells, N=32, M=32 spherical design, chunked plain passes):
    sampled cells against the oracle to 1e-12."""
    from tests.gpu_util import oracle_plan_of
    label("n32 fp64 full batch")
    f = gen.shock_batch(256, 32, 8.0, seed=2)
    col = collider(32, 256, 0, rule="design")
    q = run(col, f, f_dtype=torch.float64)
    assert np.isfinite(q).all()
    sample = [1, 100, 254]
    ref, loss = oracle_cells(f[sample], oracle_plan_of(col.plan, 32, 32))
    err = cell_errors(q[sample], ref, loss)
    assert err.max() <= 1e-12, err


@pytest.mark.parametrize("n,precision,tol,transform", [(24, 1, 1e-5, 1), (24, 1, 1e-5, 2), (24, 0, 1e-12, 0),
                                                       (48, 1, 1e-5, 0)])
def test_radix3_sizes(n, precision, tol, transform):
    import paper_2505_03360_amd as bz
    label("radix3", n, precision, transform)
    f = gen.bimaxwellian_batch(2, n, 8.0, seed=n)
    col = collider(n, 2, precision, rule="spiral", m=8, transform=transform)
    if n == 24 and transform == 1:  # fused, direction chunks from the size (four at two cells)
        assert bz.bz_plan_strategy(col.plan) == (bz.BZ_XF_FUSED, 4, 1)
    q = run(col, f)
    ref, loss = oracle_cells(f, oracle_plan(n, rule="spiral", m=8))
    err = cell_errors(q, ref, loss)
    assert err.max() <= tol, err


@pytest.mark.parametrize("n,rule,m,cells", [(16, "icosa6", 6, 5), (32, "design", 32, 3), (48, "spiral", 8, 2)])
def test_dft_gemm_against_oracle(n, rule, m, cells):
    """BZ_XF_DFT_GEMM plans (the chunked plain path with the transforms along
    k1 as FP32 MFMA products with the DFT matrix), gathered and scattered
    rows, against the oracle to the FP32 bound; the FFT plain path on the same
    cells agrees to the same bound; conservation after projection."""
    import paper_2505_03360_amd as bz
    from tests.gpu_util import oracle_plan_of
    label("dft gemm", n, rule, m)
    rows = cells + 4
    allf = gen.shock_batch(rows, n, 8.0, seed=60 + n)
    idx = np.arange(rows - 1, rows - 1 - 2 * cells, -2).astype(np.int32)
    col = collider(n, cells, 1, rule=rule, m=m, transform=bz.BZ_XF_DFT_GEMM, chunks=4)
    assert bz.bz_plan_strategy(col.plan)[:2] == (bz.BZ_XF_DFT_GEMM, 4)
    out = torch.full((rows, n, n, n), 5.0, dtype=torch.float64, device="cuda")
    q = run(col, allf, idx=idx, scatter=True, out=out)
    oplan = oracle_plan_of(col.plan, n, m) if rule == "design" else oracle_plan(n, rule=rule, m=m)
    ref, loss = oracle_cells(allf[idx], oplan)
    err = cell_errors(q[idx], ref, loss)
    print("max err", err.max(), flush=True)
    assert err.max() <= 1e-5, err
    assert np.all(q[np.setdiff1d(np.arange(rows), idx)] == 5.0)
    for c in idx:
        assert spectral.moment_drift(q[c], n, 8.0) <= 1e-12
    plain = collider(n, cells, 1, rule=rule, m=m, transform=bz.BZ_XF_PLAIN, chunks=4)
    qp = run(plain, allf[idx])
    assert cell_errors(qp, ref, loss).max() <= 1e-5


def test_n24_fused_batch_sampled():
    """N=24 on the fused kernel (one cell per workgroup, the whole 24^3 volume
    in LDS, planes that straddle waves): 300 shock cells with the spherical
    design (one chunk, projection in the epilogue), six cells against the
    oracle, every 20th cell for conservation; the same cells through the
    chunked plain path agree to the FP32 bound."""
    import paper_2505_03360_amd as bz
    from tests.gpu_util import oracle_plan_of
    label("n24 fused batch")
    f = gen.shock_batch(300, 24, 8.0, seed=24)
    col = collider(24, 300, 1, rule="design", transform=1)
    assert bz.bz_plan_strategy(col.plan) == (bz.BZ_XF_FUSED, 1, 1)
    q = run(col, f)
    assert np.isfinite(q).all()
    sample = [0, 57, 123, 199, 250, 299]
    ref, loss = oracle_cells(f[sample], oracle_plan_of(col.plan, 24, 32))
    err = cell_errors(q[sample], ref, loss)
    print("max err", err.max(), flush=True)
    assert err.max() <= 1e-5, err
    for c in range(0, 300, 20):
        assert spectral.moment_drift(q[c], 24, 8.0) <= 1e-12
    plain = collider(24, 300, 1, rule="design", transform=2)
    qp = run(plain, f)
    assert cell_errors(qp[sample], ref, loss).max() <= 1e-5


@pytest.mark.parametrize("gamma,transform", [(0.0, 1), (0.5, 2), (0.5, 1)])
def test_vhs_exponents(gamma, transform):
    label("gamma", gamma, transform)
    f = gen.shock_batch(2, 16, 8.0, seed=3)
    col = collider(16, 2, 1, rule="spiral", m=16, gamma=gamma, transform=transform)
    q = run(col, f)
    ref, loss = oracle_cells(f, oracle_plan(16, rule="spiral", m=16, gamma=gamma))
    assert cell_errors(q, ref, loss).max() <= 1e-5


@pytest.mark.parametrize("precision", [0, 1])
def test_raw_output_without_projection(precision):
    label("raw", precision)
    f = gen.bimaxwellian_batch(3, 16, 8.0, seed=4)
    col = collider(16, 3, precision, rule="product44", m=16, project=0)
    q = run(col, f, f_dtype=torch.float32 if precision else torch.float64)
    fin = f.astype(np.float32).astype(np.float64) if precision else f
    ref, loss = oracle_cells(fin, oracle_plan(16, rule="product44", m=16), project=False)
    tol = 1e-5 if precision else 1e-12
    assert cell_errors(q, ref, loss).max() <= tol


@pytest.mark.parametrize("precision,transform", [(1, 1), (0, 2)])
def test_batch_independence_bitwise(precision, transform):
    """A cell's result does not depend on the rest of the batch."""
    label("bitwise", precision, transform)
    n = 32 if transform == 1 else 16
    f = gen.shock_batch(9, n, 8.0, seed=8)
    col = collider(n, 9, precision, rule="spiral", m=8, transform=transform)
    q_all = run(col, f)
    for c in (0, 4, 8):
        q_one = run(col, f[c:c + 1])
        assert np.array_equal(q_one[0], q_all[c])
    q_rev = run(col, f[::-1].copy())
    assert np.array_equal(q_rev[::-1], q_all)


def test_device_count():
    """ncells_dev limits the processed cells on the GPU."""
    label("device count")
    f = gen.bimaxwellian_batch(8, 16, 8.0, seed=9)
    col = collider(16, 8, 1, rule="spiral", m=8)
    cnt = torch.tensor([5], dtype=torch.int32, device="cuda")
    out = torch.full((8, 16, 16, 16), -3.0, dtype=torch.float64, device="cuda")
    q = run(col, f, ncells_dev=cnt, out=out)
    full = run(col, f)
    assert np.array_equal(q[:5], full[:5])
    assert np.all(q[5:] == -3.0)


def test_timing_and_errors():
    import paper_2505_03360_amd as bz
    col = collider(16, 4, 1, rule="spiral", m=8)
    bz.bz_plan_set_timing(col.plan, True)
    f = torch.from_numpy(gen.bimaxwellian_batch(4, 16, 8.0, seed=2)).cuda()
    col(f)
    ms = bz.bz_plan_last_times(col.plan)
    assert ms[3] > 0 and all(x >= 0 for x in ms)
    with pytest.raises(bz.BzError) as e:
        col(torch.cat([f, f]))  # 8 cells > capacity 4
    assert e.value.code == bz.BZ_ERR_NOMEM


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_nonfinite_input_reported_by_sync(prec):
    import paper_2505_03360_amd as bz
    print("case numeric status", prec, flush=True)
    n = 16
    f = torch.from_numpy(gen.shock_batch(3, n, 8.0, seed=9)).cuda()
    col = bz.Collider(n, 3, L=8.0, m=6, dir_kind=bz.BZ_DIRS_ICOSA6,
                      precision=bz.BZ_FP32 if prec == "fp32" else bz.BZ_FP64)
    col(f)
    bz.bz_plan_sync(col.plan)  # finite: no error
    g = f.clone()
    g[2, 3, 4, 5] = float("nan")
    col(g)
    with pytest.raises(bz.BzError) as e:
        bz.bz_plan_sync(col.plan)
    assert e.value.code == bz.BZ_ERR_NUMERIC
    bz.bz_plan_sync(col.plan)  # the flag was cleared
    col(f)
    bz.bz_plan_sync(col.plan)
    col.close()


@pytest.mark.parametrize("n", [32, 48])
def test_maximum_request_size_sampled(n):
    # 4096 cells, the largest request of the serving workload: sampled cells against the oracle
    import paper_2505_03360_amd as bz
    print("case max size", n, flush=True)
    cells, L = 4096, 8.0
    base = gen.shock_batch(16, n, L, seed=50 + n)
    f = torch.from_numpy(base).cuda().repeat(cells // 16, 1, 1, 1).contiguous()
    f[cells - 1] = torch.from_numpy(gen.shock_batch(1, n, L, seed=99)[0]).cuda()
    col = bz.Collider(n, cells, L=L, m=32, dir_kind=bz.BZ_DIRS_SPIRAL, precision=bz.BZ_FP32)
    idx = torch.arange(cells - 1, -1, -1, dtype=torch.int32, device="cuda")  # reversed rows, scattered back
    q = torch.zeros((cells, n, n, n), dtype=torch.float64, device="cuda")
    col(f, idx=idx, out=q, scatter=True)
    torch.cuda.synchronize()
    plan = oracle_plan(n, rule="spiral", m=32)
    for r in (0, 7, cells - 1):
        fr = f[r].cpu().numpy()
        qq, _, loss = spectral.collide_fft(fr, plan, parts=True)
        err = spectral.rel_err(q[r].cpu().numpy(), spectral.project(qq, n, L), loss)
        print(f"  row {r}: err {err:.3e}", flush=True)
        assert err <= 1e-5
    assert torch.equal(q[0], q[16])  # identical inputs give identical outputs anywhere in the batch
    col.close()


@pytest.mark.parametrize("n,precision,tol,transform", [(16, 1, 1e-5, 1), (32, 1, 1e-5, 1), (16, 0, 1e-12, 2)])
def test_explicit_rule_with_a_negative_weight(n, precision, tol, transform):
    """An explicit direction rule (the 8-point spiral's directions) with
    uneven weights, one of them negative, summing to 2 pi: the fused FP32
    kernels take each direction's weight inside its multipliers (sqrt|w| on
    the real part, sign(w) sqrt|w| on the imaginary one) and the plain FP64
    path multiplies by it; both against the oracle with the same rule."""
    import paper_2505_03360_amd as bz
    from oracle import directions
    label("explicit rule, negative weight", n, precision, transform)
    d, _ = directions.spiral(8)
    c = np.array([1.8, -0.5, 1.0, 1.2, 0.5, 1.5, 1.0, 0.6])
    w = c / c.sum() * 2 * np.pi
    f = gen.bimaxwellian_batch(3, n, 8.0, seed=41)
    col = bz.Collider(n, 3, L=8.0, precision=precision, dirs=d, weights=w, transform=transform)
    assert col.transform == transform
    q = run(col, f)
    plan = spectral.Plan(n, 8.0, spectral.default_R(8.0), 1.0, 4.0, d, w)
    ref, loss = oracle_cells(f, plan)
    err = cell_errors(q, ref, loss)
    assert err.max() <= tol, err
    for i in range(3):
        assert spectral.moment_drift(q[i], n, 8.0) <= 1e-12
