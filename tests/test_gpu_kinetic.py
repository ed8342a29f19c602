"""Cell moments / L1 distance and the penalised IMEX step on the GPU against
the oracle (through the C ABI)."""
import math

import numpy as np
import pytest

import bz_inputs as gen
from oracle import kinetic, spectral
from tests.gpu_util import lib_kwargs, oracle_cells, oracle_plan

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


@pytest.mark.parametrize("n", [16, 24, 32, 48])
@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_moments_against_oracle(n, dtype):
    import paper_2505_03360_amd as bz
    print("case moments", n, dtype, flush=True)
    L = 8.0
    f = gen.shock_batch(7, n, L, seed=n)
    if dtype == "f32":
        f = f.astype(np.float32).astype(np.float64)  # the values the GPU reads
    ft = torch.from_numpy(f.astype(np.float32) if dtype == "f32" else f).cuda()
    idx = torch.tensor([5, 0, 3, 6], dtype=torch.int32, device="cuda")
    got = bz.cell_moments(ft, L, idx=idx, scatter=True)
    torch.cuda.synchronize()
    got = {k: v.cpu().numpy() for k, v in got.items()}
    for r in range(7):
        if r not in (5, 0, 3, 6):
            assert all(got[k][r] == 0.0 for k in got)  # rows not listed are not written
            continue
        rho, u, T = kinetic.moments(f[r], n, L)
        l1 = kinetic.l1_distance(f[r], n, L)
        assert abs(got["rho"][r] - rho) <= 1e-13 * rho
        assert max(abs(got["u1"][r] - u[0]), abs(got["u2"][r] - u[1]), abs(got["u3"][r] - u[2])) <= 1e-12
        assert abs(got["T"][r] - T) <= 1e-12 * T
        assert abs(got["l1"][r] - l1) <= 1e-12 * rho
    # compact output, no idx, l1 off
    got = bz.cell_moments(ft, L, l1=False)
    torch.cuda.synchronize()
    rho0 = kinetic.moments(f[0], n, L)[0]
    assert abs(float(got["rho"][0]) - rho0) <= 1e-13 * rho0 and "l1" not in got


def transport(f, n, L, seed):
    # seeded stand-in for v . grad_x f: a velocity-weighted smooth perturbation of f
    rng = np.random.default_rng(seed)
    v = spectral.velocity_nodes(n, L)
    V1, V2, V3 = np.meshgrid(v, v, v, indexing="ij")
    out = np.empty_like(f)
    for c in range(f.shape[0]):
        k = rng.uniform(-0.5, 0.5, 3)
        out[c] = (k[0] * V1 + k[1] * V2 + k[2] * V3) * f[c] * rng.uniform(0.5, 2.0)
    return out


CASES = [
    # (n, rule, m, precision, slices)
    (16, "icosa6", 6, "fp64", 0),
    (16, "icosa6", 6, "fp32", 1),
    (16, "spiral", 32, "fp32", 2),
    (24, "spiral", 32, "fp32", 0),
    (32, "spiral", 32, "fp32", 2),
    (32, "spiral", 32, "fp64", 0),
]


@pytest.mark.parametrize("n,rule,m,prec,slices", CASES)
def test_imex_euler_against_oracle(n, rule, m, prec, slices):
    import paper_2505_03360_amd as bz
    print("case imex", n, rule, m, prec, slices, flush=True)
    L, dt = 8.0, 0.01
    cells = 3
    f = gen.shock_batch(5, n, L, seed=21 + n)
    tr = transport(f, n, L, 9)
    eps_rows = np.array([0.01, 1.0, 0.003, 0.05, 1e-4])
    rows = [4, 1, 2]
    plan = oracle_plan(n, rule=rule, m=m)
    sel = f[rows]
    q_ref, loss_ref = oracle_cells(sel, plan)
    ref = np.stack([kinetic.imex_combine(sel[c], tr[rows[c]], q_ref[c], dt, eps_rows[rows[c]], L)
                    for c in range(cells)])
    kw = lib_kwargs(rule, m)
    col = bz.Collider(n, cells, L=L, precision=bz.BZ_FP32 if prec == "fp32" else bz.BZ_FP64, slices=slices, **kw)
    ft, trt = torch.from_numpy(f).cuda(), torch.from_numpy(tr).cuda()
    idx = torch.tensor(rows, dtype=torch.int32, device="cuda")
    et = torch.from_numpy(eps_rows).cuda()
    out = col.imex_euler(ft, trt, dt, eps_cells=et, idx=idx)
    torch.cuda.synchronize()
    out = out.cpu().numpy()
    tol_q = 1e-5 if prec == "fp32" else 1e-12
    for c in range(cells):
        rho1 = kinetic.conserved(sel[c] - dt * tr[rows[c]], n, L)[0]
        sens = dt / (eps_rows[rows[c]] + 2 * math.pi * rho1 * dt)  # d f^{n+1} / d Q
        qn = max(np.linalg.norm(q_ref[c]), 0.05 * np.linalg.norm(loss_ref[c]))
        err = np.linalg.norm(out[c] - ref[c])
        bound = tol_q * sens * qn + 1e-13 * np.linalg.norm(ref[c])
        print(f"  cell {c}: err {err:.3e} bound {bound:.3e}", flush=True)
        assert err <= bound
    # scalar eps, in place over the listed rows (scatter), against the same oracle
    ref2 = [kinetic.imex_combine(sel[c], tr[rows[c]], q_ref[c], dt, 0.02, L) for c in range(cells)]
    col.imex_euler(ft, trt, dt, eps=0.02, idx=idx, out=ft, scatter=True)
    torch.cuda.synchronize()
    got = ft.cpu().numpy()
    for c in range(cells):
        rho1 = kinetic.conserved(sel[c] - dt * tr[rows[c]], n, L)[0]
        sens = dt / (0.02 + 2 * math.pi * rho1 * dt)
        qn = max(np.linalg.norm(q_ref[c]), 0.05 * np.linalg.norm(loss_ref[c]))
        assert np.linalg.norm(got[rows[c]] - ref2[c]) <= tol_q * sens * qn + 1e-13 * np.linalg.norm(ref2[c])
    assert np.array_equal(got[[0, 3]], f[[0, 3]])  # rows not listed untouched
    col.close()


def test_imex_benchmarked_batch_sampled():
    """The benchmarked IMEX launch: 256 shock cells, N = 32, M = 32 spiral, FP32
    fused collision with the IMEX epilogue, v1 f as the transport term, dt = eps
    = 0.01; sampled cells against the oracle within the Q bound carried through
    the update."""
    import paper_2505_03360_amd as bz
    print("case imex 256 cells", flush=True)
    n, L, dt, eps, cells = 32, 8.0, 0.01, 0.01, 256
    f = gen.shock_batch(cells, n, L, seed=2)
    tr = f * gen.velocity_axis(n, L).reshape(1, n, 1, 1)
    col = bz.Collider(n, cells, L=L, precision=bz.BZ_FP32, **lib_kwargs("spiral", 32))
    out = col.imex_euler(torch.from_numpy(f).cuda(), torch.from_numpy(tr).cuda(), dt, eps=eps)
    torch.cuda.synchronize()
    out = out.cpu().numpy()
    assert np.isfinite(out).all()
    sample = [0, 90, 255]
    q_ref, loss_ref = oracle_cells(f[sample], oracle_plan(n, rule="spiral", m=32))
    for i, c in enumerate(sample):
        ref = kinetic.imex_combine(f[c], tr[c], q_ref[i], dt, eps, L)
        rho1 = kinetic.conserved(f[c] - dt * tr[c], n, L)[0]
        sens = dt / (eps + 2 * math.pi * rho1 * dt)
        qn = max(np.linalg.norm(q_ref[i]), 0.05 * np.linalg.norm(loss_ref[i]))
        err = np.linalg.norm(out[c] - ref)
        bound = 1e-5 * sens * qn + 1e-13 * np.linalg.norm(ref)
        print(f"  cell {c}: err {err:.3e} bound {bound:.3e}", flush=True)
        assert err <= bound
    col.close()


def test_moments_and_esbgk_benchmarked_batch_sampled():
    """The benchmarked launches of the moments and the ES-BGK operator (256 shock
    cells, N = 32, beta = -1/2, mu0 = 1): every cell's moments and sampled
    ES-BGK outputs against the oracle."""
    import paper_2505_03360_amd as bz
    print("case moments + esbgk 256 cells", flush=True)
    n, L, cells, beta, mu0 = 32, 8.0, 256, -0.5, 1.0
    f = gen.shock_batch(cells, n, L, seed=2)
    ft = torch.from_numpy(f).cuda()
    got = bz.cell_moments(ft, L)
    q = bz.esbgk_collide(ft, L, beta, mu0)
    torch.cuda.synchronize()
    got = {k: v.cpu().numpy() for k, v in got.items()}
    q = q.cpu().numpy()
    for c in range(0, cells, 17):
        rho, u, T = kinetic.moments(f[c], n, L)
        assert abs(got["rho"][c] - rho) <= 1e-13 * rho
        assert abs(got["T"][c] - T) <= 1e-12 * T
        assert abs(got["l1"][c] - kinetic.l1_distance(f[c], n, L)) <= 1e-12 * rho
    for c in (0, 128, 255):
        ref = kinetic.esbgk_collide(f[c], n, L, beta, mu0)
        rho, u, th = kinetic.stress(f[c], n, L)
        nu = kinetic.esbgk_frequency(rho, np.trace(th) / 3, beta, mu0)
        floor = max(np.linalg.norm(ref), 0.05 * nu * np.linalg.norm(f[c]))
        assert np.linalg.norm(q[c] - ref) / floor <= 1e-12


def test_imex_equilibrium_and_conservation():
    # f^n Maxwellian, no transport: f^{n+1} = f^n + dt Q(M)/(eps + beta dt) stays Maxwellian;
    # with transport the invariants of f^{n+1} are those of f^n - dt tr
    import paper_2505_03360_amd as bz
    print("case imex equilibrium", flush=True)
    n, L = 32, 8.0
    v = spectral.velocity_nodes(n, L)
    M = kinetic.maxwellian(1.0, [0.3, -0.2, 0.1], 1.0, n, L)[None]
    f = np.concatenate([M, gen.shock_batch(1, n, L, seed=3)])
    tr = transport(f, n, L, 4)
    col = bz.Collider(n, 2, L=L, precision=bz.BZ_FP32, m=32, dir_kind=bz.BZ_DIRS_SPIRAL)
    ft = torch.from_numpy(f).cuda()
    out = col.imex_euler(ft, torch.zeros_like(ft), 0.01, eps=1e-3).cpu().numpy()
    # for f = M and no transport eq. (4.24) leaves f^{n+1} - M = dt Q(M) / (eps + beta dt),
    # beta = 2 pi rho: the FP32 operator's error bar (1e-5 of the loss-floored norm) scaled
    # by the step's factor bounds the departure from equilibrium
    qq, _, ql = spectral.collide_parts(M[0], oracle_plan(n, rule="spiral", m=32))
    factor = 0.01 / (1e-3 + 2.0 * np.pi * 0.01)
    bound = factor * 1e-5 * max(np.linalg.norm(qq), 0.05 * np.linalg.norm(ql))
    assert np.linalg.norm(out[0] - M[0]) <= bound
    out = col.imex_euler(ft, torch.from_numpy(tr).cuda(), 0.01, eps=1e-3).cpu().numpy()
    for c in range(2):
        U1 = kinetic.conserved(f[c] - 0.01 * tr[c], n, L)
        assert np.abs(kinetic.conserved(out[c], n, L) - U1).max() <= 1e-6 * np.abs(U1).max()
    col.close()


@pytest.mark.parametrize("n", [16, 24, 32, 48])
@pytest.mark.parametrize("beta", [-0.5, 0.0, 0.5])
def test_esbgk_collide_against_oracle(n, beta):
    import paper_2505_03360_amd as bz
    print("case esbgk", n, beta, flush=True)
    L, mu0 = 8.0, 0.9
    f = gen.shock_batch(5, n, L, seed=40 + n)
    rows = [3, 0, 4]
    idx = torch.tensor(rows, dtype=torch.int32, device="cuda")
    q = bz.esbgk_collide(torch.from_numpy(f).cuda(), L, beta, mu0, idx=idx).cpu().numpy()
    for c, r in enumerate(rows):
        ref = kinetic.esbgk_collide(f[r], n, L, beta, mu0)
        rho, u, th = kinetic.stress(f[r], n, L)
        nu = kinetic.esbgk_frequency(rho, np.trace(th) / 3, beta, mu0)
        floor = max(np.linalg.norm(ref), 0.05 * nu * np.linalg.norm(f[r]))
        err = np.linalg.norm(q[c] - ref) / floor
        print(f"  row {r}: err {err:.3e}", flush=True)
        assert err <= 1e-12


@pytest.mark.parametrize("n", [16, 32, 48])
def test_esbgk_imex_against_oracle(n):
    import paper_2505_03360_amd as bz
    print("case esbgk imex", n, flush=True)
    L, dt, beta, mu0 = 8.0, 0.01, -0.5, 1.0
    f = gen.shock_batch(4, n, L, seed=50 + n)
    tr = transport(f, n, L, 11)
    eps_rows = np.array([0.01, 1e-4, 0.2, 3.0])
    rows = [2, 0, 3]
    ft, trt = torch.from_numpy(f).cuda(), torch.from_numpy(tr).cuda()
    idx = torch.tensor(rows, dtype=torch.int32, device="cuda")
    out = bz.esbgk_imex_euler(ft, trt, L, dt, eps_cells=torch.from_numpy(eps_rows).cuda(), beta=beta, mu0=mu0,
                              idx=idx).cpu().numpy()
    for c, r in enumerate(rows):
        ref = kinetic.esbgk_imex_euler(f[r], tr[r], dt, eps_rows[r], L, beta, mu0)
        assert np.linalg.norm(out[c] - ref) <= 1e-12 * np.linalg.norm(ref)
    # in place over the listed rows with a scalar eps
    bz.esbgk_imex_euler(ft, trt, L, dt, eps=0.05, beta=beta, mu0=mu0, idx=idx, out=ft, scatter=True)
    got = ft.cpu().numpy()
    for r in rows:
        ref = kinetic.esbgk_imex_euler(f[r], tr[r], dt, 0.05, L, beta, mu0)
        assert np.linalg.norm(got[r] - ref) <= 1e-12 * np.linalg.norm(ref)
    assert np.array_equal(got[1], f[1])


@pytest.mark.parametrize("n,rule,m,prec", [(16, "icosa6", 6, "fp64"), (16, "icosa6", 6, "fp32"),
                                           (32, "spiral", 32, "fp32"), (24, "spiral", 32, "fp32")])
def test_pr222_against_oracle(n, rule, m, prec):
    import paper_2505_03360_amd as bz
    print("case pr222", n, rule, m, prec, flush=True)
    L, dt, eps = 8.0, 0.01, 0.05
    f = gen.shock_batch(4, n, L, seed=60 + n)
    rows = [3, 1]
    v = spectral.velocity_nodes(n, L)
    V1, V2, V3 = np.meshgrid(v, v, v, indexing="ij")
    wv = 0.4 * V1 - 0.3 * V2 + 0.2 * V3  # T(y) = (c . v) y keeps the step cell-local
    plan = oracle_plan(n, rule=rule, m=m)
    ref = [kinetic.pr222_step(f[r], lambda z: wv * z, dt, eps, plan) for r in rows]
    q_ref, loss_ref = oracle_cells(f[rows], plan)
    col = bz.Collider(n, len(rows), L=L, precision=bz.BZ_FP32 if prec == "fp32" else bz.BZ_FP64,
                      **lib_kwargs(rule, m))
    ft = torch.from_numpy(f).cuda()
    wt = torch.from_numpy(wv).cuda()
    idx = torch.tensor(rows, dtype=torch.int32, device="cuda")
    out = col.pr222_step(ft, lambda z: z * wt, dt, eps=eps, idx=idx).cpu().numpy()
    tol_q = 1e-5 if prec == "fp32" else 1e-12
    for c, r in enumerate(rows):
        qn = max(np.linalg.norm(q_ref[c]), 0.05 * np.linalg.norm(loss_ref[c]))
        err = np.linalg.norm(out[r] - ref[c])
        # two evaluations of Q enter y^{n+1} with weight dt/(2 eps), and one more through Y2
        bound = 4 * tol_q * (dt / eps) * qn + 1e-13 * np.linalg.norm(ref[c])
        print(f"  row {r}: err {err:.3e} bound {bound:.3e}", flush=True)
        assert err <= bound
    col.close()


def test_pr222_benchmarked_batch_sampled():
    """The benchmarked PR(2,2,2) step (256 shock cells, N = 32, M = 32 spiral,
    FP32, zero transport, dt = eps = 0.01): sampled cells against the oracle."""
    import paper_2505_03360_amd as bz
    print("case pr222 256 cells", flush=True)
    n, L, dt, eps, cells = 32, 8.0, 0.01, 0.01, 256
    f = gen.shock_batch(cells, n, L, seed=2)
    plan = oracle_plan(n, rule="spiral", m=32)
    col = bz.Collider(n, cells, L=L, precision=bz.BZ_FP32, **lib_kwargs("spiral", 32))
    ft = torch.from_numpy(f).cuda()
    zero = torch.zeros_like(ft)
    out = col.pr222_step(ft, lambda z: zero, dt, eps=eps).cpu().numpy()
    assert np.isfinite(out).all()
    sample = [5, 250]
    q_ref, loss_ref = oracle_cells(f[sample], plan)
    for i, c in enumerate(sample):
        ref = kinetic.pr222_step(f[c], lambda z: np.zeros_like(z), dt, eps, plan)
        qn = max(np.linalg.norm(q_ref[i]), 0.05 * np.linalg.norm(loss_ref[i]))
        err = np.linalg.norm(out[c] - ref)
        bound = 4 * 1e-5 * (dt / eps) * qn + 1e-13 * np.linalg.norm(ref)
        print(f"  cell {c}: err {err:.3e} bound {bound:.3e}", flush=True)
        assert err <= bound
    col.close()


@pytest.mark.parametrize("n", [16, 32])
def test_esbgk_pr222_against_oracle(n):
    import paper_2505_03360_amd as bz
    print("case esbgk pr222", n, flush=True)
    L, dt, eps, beta, mu0 = 8.0, 0.01, 0.05, -0.5, 1.0
    f = gen.shock_batch(4, n, L, seed=80 + n)
    rows = [1, 3]
    v = spectral.velocity_nodes(n, L)
    V1, V2, V3 = np.meshgrid(v, v, v, indexing="ij")
    wv = 0.4 * V1 - 0.3 * V2 + 0.2 * V3
    ref = [kinetic.esbgk_pr222_step(f[r], lambda z: wv * z, dt, eps, L, beta, mu0) for r in rows]
    ft = torch.from_numpy(f).cuda()
    wt = torch.from_numpy(wv).cuda()
    idx = torch.tensor(rows, dtype=torch.int32, device="cuda")
    out = bz.esbgk_pr222_step(ft, lambda z: z * wt, L, dt, eps=eps, beta=beta, mu0=mu0, idx=idx).cpu().numpy()
    for c, r in enumerate(rows):
        err = np.linalg.norm(out[r] - ref[c]) / np.linalg.norm(ref[c])
        print(f"  row {r}: err {err:.3e}", flush=True)
        assert err <= 1e-12
