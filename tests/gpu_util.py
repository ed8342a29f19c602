"""Helpers shared by the GPU tests: run the library through its C ABI on
torch device memory, and evaluate the oracle on the same inputs."""
import numpy as np

from oracle import directions, spectral

RULES = {
    "icosa6": (lambda m: directions.icosa6(), 1),
    "spiral": (lambda m: directions.spiral(m), 3),
    "product44": (lambda m: directions.product(4, 4), 2),
}


def oracle_plan(n, L=8.0, R=0.0, gamma=1.0, rule="spiral", m=32, c=4.0):
    d, w = RULES[rule][0](m)
    return spectral.Plan(n, L, R if R > 0 else spectral.default_R(L), gamma, c, d, w)


def lib_kwargs(rule, m):
    import paper_2505_03360_amd as bz
    kind = {"icosa6": bz.BZ_DIRS_ICOSA6, "spiral": bz.BZ_DIRS_SPIRAL, "product44": bz.BZ_DIRS_PRODUCT}[rule]
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
