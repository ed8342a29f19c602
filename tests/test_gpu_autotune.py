"""GPU run of the autotuner on a small case: every candidate is timed and
checked against the FP64 plain path; the chosen strategy passes parity."""
import pytest

import paper_2505_03360_amd as bz

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def test_autotune_small_case(tmp_path):
    from paper_2505_03360_amd.autotune import tune_case, write_table
    print("case autotune", flush=True)
    best, rows = tune_case(16, 8, bz.BZ_FP32, 6, reps=2)
    assert len(rows) == 14 and all(r["ok"] for r in rows), rows  # m = 8: plain k in {2, 4, 8}
    write_table(str(tmp_path / "t.txt"), [(16, 8, bz.BZ_FP32, 6) + best])
    bz.bz_set_tune_table(str(tmp_path / "t.txt"))
    try:
        p = bz.bz_plan_create(bz.make_plan_desc(n=16, m=8, dir_kind=bz.BZ_DIRS_DESIGN, max_cells=6))
        assert bz.bz_plan_strategy(p)[:2] == best[:2]
        bz.bz_plan_destroy(p)
    finally:
        bz.bz_set_tune_table(None)
