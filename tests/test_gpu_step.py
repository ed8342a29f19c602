"""GPU test of the captured time step (bz_step_*): every replay of the graph
(mask -> compaction -> collision over the device-counted Boltzmann cells ->
regime feedback) matches the eager calls bit for bit, with the macro fields
changing between replays; the regimes also match the mask oracle, and one
Boltzmann cell of every replay matches the FP64 collision oracle (per-cell
error <= 1e-5 with the near-equilibrium floor, moment drift <= 1e-12)."""
import numpy as np
import pytest

import bz_inputs as gen
from oracle import mask as om
from oracle import spectral
from tests.gpu_util import oracle_plan


def check_cell_against_oracle(q, f, row, plan):
    """Q of resident row `row` against the projected FP64 oracle."""
    n = plan.n
    qq, _, ql = spectral.collide_parts(f[row].double().cpu().numpy(), plan)
    got = q[row].cpu().numpy()
    err = spectral.rel_err(got, spectral.project(qq, n, plan.L), ql)
    assert err <= 1e-5, (row, err)
    assert spectral.moment_drift(got, n, plan.L) <= 1e-12


pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def test_graph_step_replays_match_eager():
    import paper_2505_03360_amd as bz
    print("case graph step", flush=True)
    nx = ny = 40
    ncell = nx * ny
    n = 16
    rho, ux, uy, T = gen.bow_shock_field(nx, ny, step=0, seed=3)
    d = om.MaskDesc(nx=nx, ny=ny, dx=1.0 / nx, dy=1.0 / ny, eta0=1e-3, delta0=1e-4)
    eps_np = np.full((ny, nx), 1e-3)
    d.eta1 = float(np.quantile(om.indicators(d, rho, ux, uy, T, eps_np)[3], 0.85))
    md = bz.mask_desc(nx, ny, d.dx, d.dy, eta0=d.eta0, eta1=d.eta1, delta0=d.delta0)
    cu = lambda a, dt=torch.float64: torch.from_numpy(np.ascontiguousarray(a)).to("cuda", dt)
    fields = [cu(x) for x in (rho, ux, uy, T)]
    eps = cu(eps_np)
    reg_graph = torch.ones((ny, nx), dtype=torch.uint8, device="cuda")
    reg_eager = reg_graph.clone()
    reg_out = torch.empty_like(reg_graph)
    idx = torch.zeros(ncell, dtype=torch.int32, device="cuda")
    counts = torch.zeros(2, dtype=torch.int32, device="cuda")
    f = cu(np.tile(gen.bimaxwellian_batch(50, n, 8.0, seed=11), (ncell // 50 + 1, 1, 1, 1))[:ncell])
    q_graph = torch.zeros((ncell, n, n, n), dtype=torch.float64, device="cuda")
    q_eager = torch.zeros_like(q_graph)
    col = bz.Collider(n, ncell, L=8.0, m=8, dir_kind=bz.BZ_DIRS_SPIRAL, precision=bz.BZ_FP32)
    b = bz.BzStepBuffers()
    b.rho, b.ux, b.uy, b.T = [t.data_ptr() for t in fields]
    b.eps = eps.data_ptr()
    b.regime_in, b.regime_out = reg_graph.data_ptr(), reg_out.data_ptr()
    b.boltz_idx, b.counts = idx.data_ptr(), counts.data_ptr()
    b.f, b.f_dtype, b.q = f.data_ptr(), bz.BZ_FP64, q_graph.data_ptr()
    step = bz.bz_step_create(col.plan, md, b)
    stream = torch.cuda.current_stream().cuda_stream
    o_reg = np.ones((ny, nx), np.uint8)
    oplan = oracle_plan(n, rule="spiral", m=8)
    for k in range(4):
        new = gen.bow_shock_field(nx, ny, step=k, seed=3)
        for t, a in zip(fields, new):
            t.copy_(cu(a))
        torch.cuda.synchronize()
        # eager reference on its own regime state
        r2, i2, c2, _ = bz.realizability_mask(md, *fields, eps, reg_eager)
        torch.cuda.synchronize()
        cnt = int(c2[0])
        if cnt:
            col(f, idx=i2[:cnt].contiguous(), out=q_eager, scatter=True)
        reg_eager.copy_(r2)
        # graph replay
        bz.bz_step_launch(step, stream)
        torch.cuda.synchronize()
        assert int(counts[0]) == cnt and 0 < cnt < ncell
        assert torch.equal(idx[:cnt], i2[:cnt])
        assert torch.equal(reg_graph, reg_eager)
        rows = i2[:cnt].long()
        assert torch.equal(q_graph[rows], q_eager[rows])
        check_cell_against_oracle(q_graph, f, int(rows[(37 * k) % cnt]), oplan)
        # regimes against the oracle
        o_out, o_idx, _, _ = om.realizability_mask(d, *new, eps_np, o_reg)
        assert np.array_equal(reg_graph.cpu().numpy(), o_out)
        o_reg = o_out
    bz.bz_step_destroy(step)


def test_graph_step_with_kinetic_moments():
    # the captured step first recomputes the kinetic cells' fields and L1 distance from f
    import math

    import paper_2505_03360_amd as bz
    from oracle import kinetic
    print("case graph step kinetic moments", flush=True)
    nx = ny = 24
    ncell = nx * ny
    n, L = 16, 8.0
    X, Y = np.meshgrid(np.arange(nx) / nx, np.arange(ny) / ny, indexing="xy")
    rho = 1.0 + 0.05 * np.sin(2 * math.pi * X)
    T = 1.0 + 0.05 * np.cos(2 * math.pi * Y)
    ux = 0.1 * np.sin(2 * math.pi * Y)
    uy = 0.05 * np.cos(2 * math.pi * X)
    v = (np.arange(n) - n // 2) * (2 * L / n)
    V1, V2, V3 = np.meshgrid(v, v, v, indexing="ij")
    f = np.empty((ncell, n, n, n))
    for iy in range(ny):
        for ix in range(nx):
            u = [ux[iy, ix], uy[iy, ix], 0.0]
            a = 0.05 if ix >= nx // 2 else 0.0
            f[iy * nx + ix] = kinetic.maxwellian(rho[iy, ix], u, T[iy, ix], n, L) * \
                (1.0 + a * (V1 - u[0]) * (V2 - u[1]) / T[iy, ix])
    cu = lambda a, dt=torch.float64: torch.from_numpy(np.ascontiguousarray(a)).to("cuda", dt)
    # the caller's fields are deliberately off for the kinetic cells: the step recomputes them
    fields_graph = [cu(x * 1.01) for x in (rho, ux, uy, T)]
    l1_graph = torch.full((ny, nx), 1.0, dtype=torch.float64, device="cuda")
    fields_eager = [t.clone() for t in fields_graph]
    l1_eager = l1_graph.clone()
    eps = torch.full((ny, nx), 1e-4, dtype=torch.float64, device="cuda")
    reg0 = np.ones((ny, nx), np.uint8)
    reg0[:, :3] = 0  # a fluid strip keeps the caller's fields
    reg0[5:8, 15:18] = 2
    reg_graph, reg_eager = cu(reg0, torch.uint8), cu(reg0, torch.uint8)
    flags_np = np.zeros((ny, nx), np.uint8)
    flags_np[5:8, 15:18] = bz.BZ_CELL_FORCE_BOLTZMANN  # keeps a Boltzmann block for the collision stage
    flags = cu(flags_np, torch.uint8)
    reg_out = torch.empty_like(reg_graph)
    idx = torch.zeros(ncell, dtype=torch.int32, device="cuda")
    counts = torch.zeros(2, dtype=torch.int32, device="cuda")
    kin_idx = torch.zeros(ncell, dtype=torch.int32, device="cuda")
    kin_count = torch.zeros(1, dtype=torch.int32, device="cuda")
    ft = cu(f)
    q_graph = torch.zeros_like(ft)
    q_eager = torch.zeros_like(ft)
    md = bz.mask_desc(nx, ny, 1.0 / nx, 1.0 / ny, eta0=1e-3, eta1=50.0, delta0=1e-3)
    col = bz.Collider(n, ncell, L=L, m=6, dir_kind=bz.BZ_DIRS_ICOSA6, precision=bz.BZ_FP32)
    b = bz.BzStepBuffers()
    b.rho, b.ux, b.uy, b.T = [t.data_ptr() for t in fields_graph]
    b.eps, b.l1dist, b.cell_flags = eps.data_ptr(), l1_graph.data_ptr(), flags.data_ptr()
    b.regime_in, b.regime_out = reg_graph.data_ptr(), reg_out.data_ptr()
    b.boltz_idx, b.counts = idx.data_ptr(), counts.data_ptr()
    b.f, b.f_dtype, b.q = ft.data_ptr(), bz.BZ_FP64, q_graph.data_ptr()
    b.kinetic_moments, b.kin_idx, b.kin_count = 1, kin_idx.data_ptr(), kin_count.data_ptr()
    step = bz.bz_step_create(col.plan, md, b)
    stream = torch.cuda.current_stream().cuda_stream
    oplan = oracle_plan(n, rule="icosa6", m=6)
    for k in range(3):
        # eager reference: moments of the kinetic cells, mask, collision, feedback
        kin = torch.nonzero((reg_eager.view(-1) == 1) | (reg_eager.view(-1) == 2)).view(-1).int()
        out = dict(zip(("rho", "u1", "u2", "T"), [t.view(-1) for t in fields_eager]))
        out["l1"] = l1_eager.view(-1)
        if kin.numel():
            bz.cell_moments(ft, L, idx=kin, out=out, scatter=True)
        r2, i2, c2, _ = bz.realizability_mask(md, *fields_eager, eps, reg_eager, l1dist=l1_eager, cell_flags=flags)
        torch.cuda.synchronize()
        cnt = int(c2[0])
        assert cnt == 9
        if cnt:
            col(ft, idx=i2[:cnt].contiguous(), out=q_eager, scatter=True)
        reg_eager.copy_(r2)
        bz.bz_step_launch(step, stream)
        torch.cuda.synchronize()
        assert int(kin_count[0]) == kin.numel() and torch.equal(kin_idx[:kin.numel()], kin)
        for a, e in zip(fields_graph + [l1_graph], fields_eager + [l1_eager]):
            assert torch.equal(a, e)
        assert torch.equal(reg_graph, reg_eager)
        rows = i2[:cnt].long()
        assert torch.equal(q_graph[rows], q_eager[rows])
        check_cell_against_oracle(q_graph, ft, int(rows[(4 * k) % cnt]), oplan)
    # the fluid strip kept the caller's fields; near-equilibrium kinetic cells went to the fluid layer
    assert torch.equal(fields_graph[0][:, :3], cu(rho * 1.01)[:, :3])
    final = reg_graph.cpu().numpy()
    assert (final[:, 3: nx // 2] == 0).any() and (final[:, nx // 2:] >= 1).all()
    bz.bz_step_destroy(step)
