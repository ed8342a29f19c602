"""The tune table steers bz_plan_create (host only, no GPU needed)."""
import pytest

import paper_2505_03360_amd as bz
from paper_2505_03360_amd.autotune import candidates, write_table


def test_tune_table_selects_strategy(tmp_path):
    path = tmp_path / "tune.txt"
    write_table(str(path), [(16, 8, bz.BZ_FP32, 1, bz.BZ_XF_FUSED, 4, 2, 10.0),
                            (16, 8, bz.BZ_FP32, 64, bz.BZ_XF_FUSED, 1, 1, 2.0),
                            (32, 8, bz.BZ_FP32, 16, bz.BZ_XF_PLAIN, 1, 0, 50.0)])
    bz.bz_set_tune_table(str(path))
    try:
        def strategy(n, cells, **kw):
            p = bz.bz_plan_create(bz.make_plan_desc(n=n, m=8, dir_kind=bz.BZ_DIRS_SPIRAL, max_cells=cells, **kw))
            s = bz.bz_plan_strategy(p)
            bz.bz_plan_destroy(p)
            return s
        assert strategy(16, 1) == (bz.BZ_XF_FUSED, 4, 2)
        assert strategy(16, 32) == (bz.BZ_XF_FUSED, 4, 2)      # largest tuned size <= 32
        assert strategy(16, 500) == (bz.BZ_XF_FUSED, 1, 1)
        assert strategy(32, 1)[0] == bz.BZ_XF_PLAIN             # smallest entry when none fits
        assert strategy(16, 64, chunks=2) == (bz.BZ_XF_FUSED, 2, 2)  # explicit knobs win
        assert strategy(24, 64)[0] == bz.BZ_XF_FUSED            # no line for n = 24: heuristics
        assert strategy(32, 16)[:2] == (bz.BZ_XF_PLAIN, 1)       # plain: chunks = directions per launch
    finally:
        bz.bz_set_tune_table(None)
    # without a table ("") the plan sizes its direction chunks from max_cells
    bz.bz_set_tune_table("")
    try:
        for n, cells, chunks, slices in [(16, 1, 4, 2), (16, 256, 4, 2), (16, 512, 2, 2), (16, 2048, 1, 2),
                                         (24, 64, 4, 1), (24, 300, 1, 1), (32, 64, 4, 2), (32, 128, 2, 2),
                                         (32, 256, 1, 2)]:
            p = bz.bz_plan_create(bz.make_plan_desc(n=n, m=8, dir_kind=bz.BZ_DIRS_SPIRAL, max_cells=cells))
            assert bz.bz_plan_strategy(p) == (bz.BZ_XF_FUSED, chunks, slices), (n, cells)
            bz.bz_plan_destroy(p)
        for n, prec, cells, k in [(48, bz.BZ_FP32, 1024, 8), (48, bz.BZ_FP32, 4096, 4), (48, bz.BZ_FP64, 64, 4),
                                  (32, bz.BZ_FP64, 64, 8)]:
            p = bz.bz_plan_create(bz.make_plan_desc(n=n, m=8, dir_kind=bz.BZ_DIRS_SPIRAL, max_cells=cells,
                                                    precision=prec))
            assert bz.bz_plan_strategy(p)[:2] == (bz.BZ_XF_PLAIN, k), (n, prec, cells)
            bz.bz_plan_destroy(p)
    finally:
        bz.bz_set_tune_table(None)


def test_plain_directions_per_launch_knob():
    for k in (1, 2, 5, 8, 17):
        p = bz.bz_plan_create(bz.make_plan_desc(n=48, m=32, dir_kind=bz.BZ_DIRS_SPIRAL, max_cells=16, chunks=k,
                                                transform=bz.BZ_XF_PLAIN))
        tb, fixed, per = bz.bz_plan_device_bytes(p)
        assert bz.bz_plan_strategy(p)[:2] == (bz.BZ_XF_PLAIN, k)
        bz.bz_plan_destroy(p)
        assert per >= k * 48 ** 3 * 8  # k stage-A volumes of complex FP32 per cell


def test_shipped_table_is_read_by_default():
    """The library reads tune_gfx950.txt beside libbz.so when no table is set:
    every line parses, and a plan at a tuned size resolves to the line's
    strategy."""
    import os
    path = os.path.join(os.path.dirname(bz.LIB_PATH), "tune_gfx950.txt")
    if not os.path.exists(path):
        return
    lines = [ln.split() for ln in open(path) if ln.strip() and not ln.startswith("#")]
    assert lines and all(ln[0] == "gfx950" and len(ln) == 9 for ln in lines)
    bz.bz_set_tune_table(None)
    for ln in lines:
        n, m, prec, cells, x, c, s = (int(v) for v in ln[1:8])
        p = bz.bz_plan_create(bz.make_plan_desc(n=n, m=m, dir_kind=bz.BZ_DIRS_DESIGN, max_cells=cells,
                                                precision=prec))
        got = bz.bz_plan_strategy(p)
        bz.bz_plan_destroy(p)
        assert got[0] == x and got[1] == c and (x == bz.BZ_XF_PLAIN or got[2] == s), (ln, got)


def test_candidate_set():
    plain = [(bz.BZ_XF_PLAIN, k, 0) for k in (2, 4, 8, 11, 17)]
    gemm = [(bz.BZ_XF_DFT_GEMM, k, 0) for k in (2, 4, 8)]
    c16 = candidates(16, 32, bz.BZ_FP32)
    assert c16[:8] == plain + gemm and (bz.BZ_XF_FUSED, 8, 1) in c16 and len(c16) == 16
    assert candidates(24, 32, bz.BZ_FP32) == plain + [(bz.BZ_XF_FUSED, c, 1) for c in (1, 2, 4, 8)]
    assert candidates(48, 32, bz.BZ_FP32) == plain + gemm
    assert candidates(32, 32, bz.BZ_FP64) == plain


def test_dft_gemm_plans():
    """BZ_XF_DFT_GEMM: FP32 plans at n in {16, 32, 48}; the plan's tables grow
    by the matrix-core operand fragments of the inverse DFT."""
    for n in (16, 32, 48):
        p = bz.bz_plan_create(bz.make_plan_desc(n=n, m=8, dir_kind=bz.BZ_DIRS_SPIRAL, max_cells=16,
                                                transform=bz.BZ_XF_DFT_GEMM, chunks=4))
        q = bz.bz_plan_create(bz.make_plan_desc(n=n, m=8, dir_kind=bz.BZ_DIRS_SPIRAL, max_cells=16,
                                                transform=bz.BZ_XF_PLAIN, chunks=4))
        try:
            assert bz.bz_plan_strategy(p)[:2] == (bz.BZ_XF_DFT_GEMM, 4)
            tp, fp, pp = bz.bz_plan_device_bytes(p)
            tq, fq, pq = bz.bz_plan_device_bytes(q)
            assert tp - tq == -(-2 * (n // 16) * (n // 2) * 64 * 4 // 256) * 256 and (fp, pp) == (fq, pq)
        finally:
            bz.bz_plan_destroy(p)
            bz.bz_plan_destroy(q)
    for kw in (dict(n=24), dict(n=32, precision=bz.BZ_FP64)):
        with pytest.raises(bz.BzError) as e:
            bz.bz_plan_create(bz.make_plan_desc(m=8, dir_kind=bz.BZ_DIRS_SPIRAL, transform=bz.BZ_XF_DFT_GEMM, **kw))
        assert e.value.code == bz.BZ_ERR_UNSUPPORTED
