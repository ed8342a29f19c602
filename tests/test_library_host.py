"""Host-side checks of the HIP library that need no GPU: the shared object
loads and exports every entry point include/bz.h declares, descriptors are
validated, and the plan's FP64 direction rules and multiplier tables (the
library's own special functions) agree with the oracle's independent ones."""
import math
import os
import re

import numpy as np
import pytest

import paper_2505_03360_amd as bz
from oracle import directions, spectral

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_symbols():
    names = set()
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if fn.endswith(".h"):
            txt = open(os.path.join(ROOT, "include", fn)).read()
            txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
            names |= set(re.findall(r"\b(bz_[a-z0-9_]+)\s*\(", txt))
    return names


def test_library_exports_every_declared_symbol():
    L = bz.lib()
    syms = header_symbols()
    assert "bz_collide_batch" in syms and "bz_realizability_mask" in syms
    for s in sorted(syms):
        assert hasattr(L, s), s
    assert bz.bz_abi_version() == bz.ABI_VERSION
    declared = {name for name, _, _ in bz.SIGNATURES}
    assert syms <= declared, syms - declared


@pytest.mark.parametrize("kw,code", [
    (dict(n=20), bz.BZ_ERR_UNSUPPORTED),
    (dict(R=7.3), bz.BZ_ERR_ARG),
    (dict(gamma=1.5), bz.BZ_ERR_ARG),
    (dict(m=7, dir_kind=bz.BZ_DIRS_ICOSA6), bz.BZ_ERR_ARG),
    (dict(m=16, dir_kind=bz.BZ_DIRS_PRODUCT, a1=4, a2=3), bz.BZ_ERR_ARG),
    (dict(max_cells=0), bz.BZ_ERR_ARG),
    (dict(n=48, transform=bz.BZ_XF_FUSED), bz.BZ_ERR_UNSUPPORTED),
    (dict(n=24, transform=bz.BZ_XF_FUSED, slices=2), bz.BZ_ERR_UNSUPPORTED),
    (dict(precision=bz.BZ_FP64, transform=bz.BZ_XF_FUSED), bz.BZ_ERR_UNSUPPORTED),
])
def test_plan_validation(kw, code):
    args = dict(n=16, L=8.0, m=6, dir_kind=bz.BZ_DIRS_ICOSA6)
    args.update(kw)
    with pytest.raises(bz.BzError) as e:
        bz.bz_plan_create(bz.make_plan_desc(**args))
    assert e.value.code == code
    assert bz.bz_last_error() != ""


def test_explicit_rule_weight_sum_checked():
    d, w = directions.spiral(8)
    with pytest.raises(bz.BzError):
        bz.bz_plan_create(bz.make_plan_desc(n=16, dirs=d, weights=w * 1.001))
    with pytest.raises(bz.BzError):
        bz.bz_plan_create(bz.make_plan_desc(n=16, dirs=d * 1.01, weights=w))


@pytest.mark.parametrize("kind,m,a", [(bz.BZ_DIRS_ICOSA6, 6, (0, 0)), (bz.BZ_DIRS_PRODUCT, 16, (4, 4)),
                                      (bz.BZ_DIRS_SPIRAL, 32, (0, 0))])
def test_direction_rules_match_oracle(kind, m, a):
    p = bz.bz_plan_create(bz.make_plan_desc(n=16, m=m, dir_kind=kind, a1=a[0], a2=a[1]))
    d, w = bz.bz_plan_get_rule(p, m)
    bz.bz_plan_destroy(p)
    ref = {bz.BZ_DIRS_ICOSA6: directions.icosa6, bz.BZ_DIRS_PRODUCT: lambda: directions.product(4, 4),
           bz.BZ_DIRS_SPIRAL: lambda: directions.spiral(32)}[kind]()
    assert np.abs(d - ref[0]).max() <= 1e-15 and np.abs(w - ref[1]).max() <= 1e-15


@pytest.mark.parametrize("n,gamma,R", [(16, 1.0, 0.0), (16, 0.0, 5.0), (24, 0.5, 0.0), (32, 1.0, 7.2)])
def test_multipliers_match_oracle(n, gamma, R):
    L = 8.0
    p = bz.bz_plan_create(bz.make_plan_desc(n=n, L=L, R=R, gamma=gamma, m=32, dir_kind=bz.BZ_DIRS_SPIRAL))
    d, w = directions.spiral(32)
    plan = spectral.Plan(n, L, R if R > 0 else spectral.default_R(L), gamma, 4.0, d, w)
    for pi in (0, 7, 31):
        a, ap = bz.bz_plan_get_multipliers(p, n, pi)
        ra, rap = spectral.multipliers(plan, pi)
        assert np.abs(a - ra).max() <= 1e-12 * np.abs(ra).max(), pi
        assert np.abs(ap - rap).max() <= 1e-12 * np.abs(rap).max(), pi
    bl, one = bz.bz_plan_get_multipliers(p, n, 32)
    assert np.abs(bl - spectral.bhat_m(plan)).max() <= 1e-12 * np.abs(bl).max()
    assert np.all(one == 1.0)
    bz.bz_plan_destroy(p)


def test_device_bytes_scale():
    p = bz.bz_plan_create(bz.make_plan_desc(n=32, m=32, dir_kind=bz.BZ_DIRS_SPIRAL, precision=bz.BZ_FP32))
    t, fixed, per = bz.bz_plan_device_bytes(p)
    assert t >= 33 * 32 ** 3 * 8
    assert per >= 32 ** 3 * (8 + 4)  # fhat (complex FP32) and the FP32 copy of f; the rest stays on chip
    assert bz.bz_plan_transform(p) == bz.BZ_XF_FUSED
    with pytest.raises(bz.BzError) as e:
        bz.bz_plan_capacity(p)
    assert e.value.code == bz.BZ_ERR_STATE
    bz.bz_plan_destroy(p)
    p = bz.bz_plan_create(bz.make_plan_desc(n=32, m=32, dir_kind=bz.BZ_DIRS_SPIRAL, precision=bz.BZ_FP64))
    assert bz.bz_plan_transform(p) == bz.BZ_XF_PLAIN
    assert bz.bz_plan_device_bytes(p)[2] >= 32 ** 3 * (16 + 16 + 8)  # fhat, scratch volume, accumulator
    bz.bz_plan_destroy(p)


def test_moments_and_imex_validation():
    out = bz.BzMomentsOut()
    with pytest.raises(bz.BzError) as e:
        bz.bz_cell_moments(20, 8.0, 0, bz.BZ_FP64, 0, 4, 0, out)
    assert e.value.code == bz.BZ_ERR_UNSUPPORTED
    with pytest.raises(bz.BzError) as e:
        bz.bz_cell_moments(32, 0.0, 0, bz.BZ_FP64, 0, 4, 0, out)
    assert e.value.code == bz.BZ_ERR_ARG
    with pytest.raises(bz.BzError) as e:
        bz.bz_cell_moments(32, 8.0, 0, bz.BZ_FP64, 0, 4, 0, out, flags=bz.BZ_SCATTER)
    assert e.value.code == bz.BZ_ERR_ARG
    bz.bz_cell_moments(32, 8.0, 0, bz.BZ_FP64, 0, 0, 0, out)  # empty batch: nothing to do
    p = bz.bz_plan_create(bz.make_plan_desc(n=16, m=6, precision=bz.BZ_FP64))
    with pytest.raises(bz.BzError) as e:
        bz.bz_imex_euler(p, bz.BzImexDesc(0.01, 0.1, None), 0, 0, 0, 1, 0, 0)
    assert e.value.code == bz.BZ_ERR_STATE  # not bound
    bz.bz_plan_destroy(p)


def test_esbgk_validation():
    imex = bz.BzImexDesc(0.01, 0.1, None)
    for desc, code in ((bz.BzEsbgkDesc(20, 8.0, -0.5, 1.0), bz.BZ_ERR_UNSUPPORTED),
                       (bz.BzEsbgkDesc(32, 8.0, 1.0, 1.0), bz.BZ_ERR_ARG),
                       (bz.BzEsbgkDesc(32, 8.0, -0.5, 0.0), bz.BZ_ERR_ARG),
                       (bz.BzEsbgkDesc(32, -1.0, -0.5, 1.0), bz.BZ_ERR_ARG)):
        with pytest.raises(bz.BzError) as e:
            bz.bz_esbgk_collide(desc, 0, 0, 4, 0, 0)
        assert e.value.code == code
        with pytest.raises(bz.BzError) as e:
            bz.bz_esbgk_imex_euler(desc, imex, 0, 0, 0, 4, 0, 0)
        assert e.value.code == code
    good = bz.BzEsbgkDesc(32, 8.0, -0.5, 1.0)
    with pytest.raises(bz.BzError) as e:
        bz.bz_esbgk_imex_euler(good, bz.BzImexDesc(0.0, 0.1, None), 0, 0, 0, 4, 0, 0)
    assert e.value.code == bz.BZ_ERR_ARG
    with pytest.raises(bz.BzError) as e:
        bz.bz_esbgk_collide(good, 0, 0, 4, 0, 0)  # null pointers
    assert e.value.code == bz.BZ_ERR_ARG
    bz.bz_esbgk_collide(good, 0, 0, 0, 0, 0)  # empty batch


def test_pr222_validation():
    p = bz.bz_plan_create(bz.make_plan_desc(n=16, m=6, precision=bz.BZ_FP64))
    d = bz.BzImexDesc(0.01, 0.1, None)
    for fn, args in ((bz.bz_pr222_stage1, (0, 0, 1, 0, 0)), (bz.bz_pr222_stage2, (0, 0, 0, 0, 1, 0, 0, 0)),
                     (bz.bz_pr222_finish, (0, 0, 0, 0, 1, 0, 0))):
        with pytest.raises(bz.BzError) as e:
            fn(p, d, *args)
        assert e.value.code == bz.BZ_ERR_STATE  # not bound
    bz.bz_plan_destroy(p)


def test_dealias_plans():
    with pytest.raises(bz.BzError) as e:
        bz.bz_plan_create(bz.make_plan_desc(n=24, m=6, dealias=1))
    assert e.value.code == bz.BZ_ERR_UNSUPPORTED
    with pytest.raises(bz.BzError) as e:
        bz.bz_plan_create(bz.make_plan_desc(n=16, m=6, dealias=2))
    assert e.value.code == bz.BZ_ERR_ARG
    p = bz.bz_plan_create(bz.make_plan_desc(n=16, m=6, dealias=1, precision=bz.BZ_FP64))
    q = bz.bz_plan_create(bz.make_plan_desc(n=24, m=6, precision=bz.BZ_FP64, project=0))
    tp, _, wp = bz.bz_plan_device_bytes(p)
    tq, _, wq = bz.bz_plan_device_bytes(q)
    assert tp == tq  # the device tables are the padded operator's
    assert wp > wq  # its workspace holds the padded plan's plus the resampling buffers
    assert bz.bz_plan_transform(p) == bz.BZ_XF_PLAIN
    bz.bz_plan_destroy(p)
    bz.bz_plan_destroy(q)


def test_esbgk_pr222_validation():
    d, im = bz.BzEsbgkDesc(32, 8.0, -0.5, 1.0), bz.BzImexDesc(0.01, 0.1, None)
    for fn, args in ((bz.bz_esbgk_pr222_stage1, (0, 0, 1, 0, 0)), (bz.bz_esbgk_pr222_stage2, (0, 0, 0, 0, 1, 0, 0, 0)),
                     (bz.bz_esbgk_pr222_finish, (0, 0, 0, 0, 1, 0, 0))):
        with pytest.raises(bz.BzError) as e:
            fn(d, im, *args)
        assert e.value.code == bz.BZ_ERR_ARG  # null arrays
        with pytest.raises(bz.BzError) as e:
            fn(d, bz.BzImexDesc(-1.0, 0.1, None), *args)
        assert e.value.code == bz.BZ_ERR_ARG  # dt <= 0


# ---------------------------------------------------------------- two velocity dimensions
@pytest.mark.parametrize("kw,code", [
    (dict(n=24), bz.BZ_ERR_UNSUPPORTED),                      # n not in {16, 32, 64}
    (dict(n=64, precision=bz.BZ_FP64), bz.BZ_ERR_UNSUPPORTED),
    (dict(gamma=1.0), bz.BZ_ERR_UNSUPPORTED),                 # Maxwell molecules only
    (dict(dir_kind=bz.BZ_DIRS_SPIRAL), bz.BZ_ERR_ARG),
    (dict(transform=bz.BZ_XF_PLAIN), bz.BZ_ERR_UNSUPPORTED),
    (dict(dealias=1), bz.BZ_ERR_ARG),
    (dict(chunks=2), bz.BZ_ERR_ARG),
    (dict(R=10.0), bz.BZ_ERR_ARG),                            # beyond 4L/(3+sqrt2)
    (dict(m=0), bz.BZ_ERR_ARG),
    (dict(dim=5), bz.BZ_ERR_ARG),
])
def test_plan2d_validation(kw, code):
    args = dict(n=32, L=8.0, gamma=0.0, kernel_c=1.0, m=16, dir_kind=bz.BZ_DIRS_CIRCLE, dim=2)
    args.update(kw)
    with pytest.raises(bz.BzError) as e:
        bz.bz_plan_create(bz.make_plan_desc(**args))
    assert e.value.code == code


def test_circle_rule_refused_in_three_dimensions():
    with pytest.raises(bz.BzError) as e:
        bz.bz_plan_create(bz.make_plan_desc(n=16, m=8, dir_kind=bz.BZ_DIRS_CIRCLE))
    assert e.value.code == bz.BZ_ERR_ARG


@pytest.mark.parametrize("n,m,R", [(16, 8, 0.0), (32, 24, 5.5), (64, 5, 0.0)])
def test_plan2d_tables_match_oracle(n, m, R):
    from oracle import maxwell2d as m2
    L = 7.0
    p = bz.bz_plan_create(bz.make_plan2d_desc(n, L=L, R=R, kernel_c=1.7, m=m))
    plan = m2.make_plan(n, L, R=R if R > 0 else None, A=m, kernel_c=1.7)
    for q in (0, m // 2, m - 1):
        a, b = bz.bz_plan_get_multipliers(p, n, q, dim=2)
        ra, rb = m2.multipliers(plan, q)
        assert np.abs(a - ra).max() <= 1e-13 * np.abs(ra).max()
        assert np.abs(b - rb).max() <= 1e-13 * np.abs(rb).max()
    bl, one = bz.bz_plan_get_multipliers(p, n, m, dim=2)
    assert np.abs(bl - m2.bhat_m(plan)).max() <= 1e-13 * np.abs(bl).max()
    assert np.all(one == 1.0)
    d, w = bz.bz_plan_get_rule(p, m)
    th = math.pi * np.arange(1, m + 1) / m
    assert np.abs(d[:, 0] - np.cos(th)).max() <= 1e-15 and np.abs(d[:, 1] - np.sin(th)).max() <= 1e-15
    assert np.all(d[:, 2] == 0.0) and abs(w.sum() - math.pi) <= 1e-13
    assert bz.bz_plan_transform(p) == bz.BZ_XF_FUSED
    t, fixed, per = bz.bz_plan_device_bytes(p)
    assert t >= (m + 1) * n * n * 8 and per > 0
    bz.bz_plan_destroy(p)


def test_plan2d_refused_by_three_dimensional_entry_points():
    p = bz.bz_plan_create(bz.make_plan2d_desc(16, m=4))
    d = bz.BzImexDesc(0.01, 0.1, None)
    with pytest.raises(bz.BzError) as e:
        bz.bz_imex_euler(p, d, 1, 1, 0, 1, 0, 1, 0, 0)
    assert e.value.code == bz.BZ_ERR_UNSUPPORTED
    with pytest.raises(bz.BzError) as e:
        bz.bz_pr222_stage1(p, d, 1, 0, 1, 0, 2, 0)
    assert e.value.code == bz.BZ_ERR_UNSUPPORTED
    bz.bz_plan_destroy(p)


@pytest.mark.parametrize("m,t", [(32, 9), (64, 15), (6, 3)])
def test_design_rule_is_a_spherical_design(m, t):
    """BZ_DIRS_DESIGN: equal weights 2 pi / m, unit vectors on the upper half
    sphere, and the antipodal design degree the library reports equals the
    one the oracle's own test (Legendre sums of the pair kernel) finds; the
    library's table agrees with the oracle's independent generator."""
    p = bz.bz_plan_create(bz.make_plan_desc(n=16, L=8.0, m=m, dir_kind=bz.BZ_DIRS_DESIGN))
    try:
        d, w = bz.bz_plan_get_rule(p, m)
        assert bz.bz_plan_rule_degree(p) == t
    finally:
        bz.bz_plan_destroy(p)
    assert np.allclose(w, 2 * math.pi / m, rtol=0, atol=1e-15)
    assert np.allclose(np.linalg.norm(d, axis=1), 1.0, rtol=0, atol=1e-14)
    assert (d[:, 2] >= 0).all()
    assert directions.design_degree(d, w) == t
    od, ow, ot = directions.design(m)
    assert ot == t and np.abs(od - d).max() <= 1e-10


def test_spiral_and_product_rules_report_degree_one():
    for kw in (dict(m=32, dir_kind=bz.BZ_DIRS_SPIRAL), dict(m=16, dir_kind=bz.BZ_DIRS_PRODUCT, a1=4, a2=4)):
        p = bz.bz_plan_create(bz.make_plan_desc(n=16, L=8.0, **kw))
        try:
            assert bz.bz_plan_rule_degree(p) == 1
        finally:
            bz.bz_plan_destroy(p)


def test_noalloc_refuses_beyond_the_static_array():
    """bz_collide_batch_noalloc checks the workspace a call needs against its
    64 MiB static array on the host, before anything touches the device (the
    plan here is not even bound; the pointers are never dereferenced)."""
    p = bz.bz_plan_create(bz.make_plan_desc(n=32, L=8.0, m=8, dir_kind=bz.BZ_DIRS_SPIRAL, precision=bz.BZ_FP64,
                                            max_cells=64))
    try:
        tb, fixed, per = bz.bz_plan_device_bytes(p)
        fits = ((64 << 20) - fixed) // per
        with pytest.raises(bz.BzError) as e:
            bz.bz_collide_batch_noalloc(p, 1 << 20, bz.BZ_FP64, 0, fits + 1, 0, 1 << 20, 0, 0)
        assert e.value.code == bz.BZ_ERR_NOMEM and f"at most {fits} cells" in str(e.value)
        with pytest.raises(bz.BzError) as e:  # within the limit: refused only because the tables are not bound
            bz.bz_collide_batch_noalloc(p, 1 << 20, bz.BZ_FP64, 0, fits, 0, 1 << 20, 0, 0)
        assert e.value.code == bz.BZ_ERR_STATE
    finally:
        bz.bz_plan_destroy(p)
