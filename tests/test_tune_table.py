"""The tune table steers bz_plan_create (host only, no GPU needed)."""
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
        assert strategy(24, 64)[0] == bz.BZ_XF_PLAIN            # no fused kernel for n = 24
    finally:
        bz.bz_set_tune_table(None)
    # without a table the plan sizes its direction chunks from max_cells
    for n, cells, chunks in [(16, 1, 4), (16, 256, 4), (16, 512, 2), (16, 2048, 1),
                             (32, 64, 4), (32, 128, 2), (32, 256, 1)]:
        p = bz.bz_plan_create(bz.make_plan_desc(n=n, m=8, dir_kind=bz.BZ_DIRS_SPIRAL, max_cells=cells))
        assert bz.bz_plan_strategy(p) == (bz.BZ_XF_FUSED, chunks, 2), (n, cells)
        bz.bz_plan_destroy(p)


def test_candidate_set():
    c16 = candidates(16, 32, bz.BZ_FP32)
    assert (bz.BZ_XF_PLAIN, 1, 0) in c16 and (bz.BZ_XF_FUSED, 8, 1) in c16 and len(c16) == 9
    assert candidates(24, 32, bz.BZ_FP32) == [(bz.BZ_XF_PLAIN, 1, 0)]
    assert candidates(32, 32, bz.BZ_FP64) == [(bz.BZ_XF_PLAIN, 1, 0)]
