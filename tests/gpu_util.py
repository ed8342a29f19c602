"""Helpers shared by the GPU tests: run the library through its C ABI on
torch device memory, and evaluate the oracle on the same inputs."""
import numpy as np

from oracle import directions, spectral

RULES = {
    "icosa6": (lambda m: directions.icosa6(), 1),
    "spiral": (lambda m: directions.spiral(m), 3),
    "product44": (lambda m: directions.product(4, 4), 2),
    "design": (lambda m: directions.design(m)[:2], 5),
}


def oracle_plan(n, L=8.0, R=0.0, gamma=1.0, rule="spiral", m=32, c=4.0):
    d, w = RULES[rule][0](m)
    return spectral.Plan(n, L, R if R > 0 else spectral.default_R(L), gamma, c, d, w)


def lib_kwargs(rule, m):
    import paper_2505_03360_amd as bz
    kind = {"icosa6": bz.BZ_DIRS_ICOSA6, "spiral": bz.BZ_DIRS_SPIRAL, "product44": bz.BZ_DIRS_PRODUCT,
            "design": bz.BZ_DIRS_DESIGN}[rule]
    kw = dict(m=m, dir_kind=kind)
    if rule == "product44":
        kw.update(a1=4, a2=4, m=16)
    return kw


def oracle_cells(f, plan, project=True):
    """Per cell: (Q projected or raw, loss) from the oracle."""
    out, loss = [], []
    for c in range(f.shape[0]):
        q, qp, ql = spectral.collide_parts(f[c], plan)
        out.append(spectral.project(q, plan.n, plan.L) if project else q)
        loss.append(ql)
    return np.stack(out), np.stack(loss)


def cell_errors(q_gpu, q_ref, loss_ref):
    return np.array([spectral.rel_err(q_gpu[c], q_ref[c], loss_ref[c]) for c in range(q_ref.shape[0])])


def oracle_loss_norms(f, plan):
    """Per cell ||C fN Lambda||_2, the loss term of the oracle (fN the truncated
    series of f, Lambda = IDFT(Bhat_M fhat)): the near-equilibrium floor of
    the per-cell error is 0.05 times it."""
    n, L = plan.n, plan.L
    bh = spectral.bhat_m(plan)
    out = np.empty(f.shape[0])
    for c in range(f.shape[0]):
        fh = spectral.forward(f[c], n, L)
        loss = spectral.inverse(fh, n, L).real * spectral.inverse(bh * fh, n, L).real
        out[c] = plan.kernel_c * np.linalg.norm(loss)
    return out


def floored_errors(q_test, q_ref, loss_norms):
    """Per-cell ||dQ|| / max(||Q_ref||, 0.05 ||loss||) and the number of cells
    where the floor binds (cancellation-dominated cells)."""
    d = np.linalg.norm((q_test - q_ref).reshape(q_ref.shape[0], -1), axis=1)
    r = np.linalg.norm(q_ref.reshape(q_ref.shape[0], -1), axis=1)
    floor = 0.05 * loss_norms
    return d / np.maximum(r, floor), int(np.sum(floor > r))


def oracle_plan_of(plan_handle, n, m, L=8.0, R=0.0, gamma=1.0, c=4.0):
    """Oracle plan on the direction table of a library plan, taken as data
    (both sides must integrate with the same rule).  A spherical-design table
    is first checked by the oracle's own degree test against the degree the
    library reports."""
    import paper_2505_03360_amd as bz
    d, w = bz.bz_plan_get_rule(plan_handle, m)
    t = bz.bz_plan_rule_degree(plan_handle)
    assert directions.design_degree(d, w) == t
    assert abs(w.sum() - 2 * np.pi) <= 1e-12 and np.allclose(np.linalg.norm(d, axis=1), 1.0, atol=1e-14)
    return spectral.Plan(n, L, R if R > 0 else spectral.default_R(L), gamma, c, d, w)
