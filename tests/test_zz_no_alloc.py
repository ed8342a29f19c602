"""GPU test of bz_collide_batch_noalloc, the evaluation whose workspace is the
library's static device array: through the C ABI, on plans bound to their
tables only, its output equals bz_collide_batch's on a plan with a bound
workspace (same descriptor, so the same strategy and arithmetic: bit for
bit), on two calls in a row, the second smaller, for the fused, multi-chunk,
chunked plain FP32 and FP64 paths; a request beyond the static array is
refused before any launch."""
import numpy as np
import pytest

import bz_inputs as gen

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


CASES = [
    # (n, max_cells, descriptor, first call cells, second call cells)
    (32, 64, dict(m=32, dir_kind=5, precision=1), 40, 12),    # fused, 4 chunks (<= 64 cells), design rule
    (32, 256, dict(m=32, dir_kind=5, precision=1), 150, 30),  # fused, one chunk, projection epilogue
    (16, 300, dict(m=6, dir_kind=1, precision=1), 150, 17),   # fused n = 16, two chunks
    (24, 40, dict(m=8, dir_kind=3, precision=1), 30, 7),      # chunked plain FP32
    (32, 12, dict(m=8, dir_kind=3, precision=0), 10, 3),      # chunked plain FP64
]


@pytest.mark.parametrize("n,cap,kw,c1,c2", CASES)
def test_noalloc_matches_bound_workspace(n, cap, kw, c1, c2):
    import paper_2505_03360_amd as bz
    print("case noalloc", n, cap, kw, c1, c2, flush=True)
    col = bz.Collider(n, cap, L=8.0, **kw)
    p = bz.bz_plan_create(bz.make_plan_desc(n=n, L=8.0, max_cells=cap, **kw))
    try:
        tb, fixed, per = bz.bz_plan_device_bytes(p)
        assert fixed + per * c1 <= 64 << 20
        tables = torch.empty(max(tb, 256), dtype=torch.uint8, device="cuda")
        stream = torch.cuda.current_stream().cuda_stream
        bz.bz_plan_bind(p, tables.data_ptr(), 0, 0, stream)
        assert bz.bz_plan_capacity(p) == 0
        assert bz.bz_plan_strategy(p) == bz.bz_plan_strategy(col.plan)
        rows = 2 * c1 + 3
        f = torch.from_numpy(gen.bimaxwellian_batch(rows, n, 8.0, seed=n + c1)).cuda()
        rng = np.random.default_rng(c1)
        # call 1: c1 cells gathered by an index list and scattered back
        idx = torch.from_numpy(np.sort(rng.choice(rows, size=c1, replace=False)).astype(np.int32)).cuda()
        ref = col(f, idx=idx, scatter=True, out=torch.full((rows, n, n, n), 3.0, dtype=col.out_dtype,
                                                            device="cuda"))
        got = torch.full_like(ref, 3.0)
        bz.bz_collide_batch_noalloc(p, f.data_ptr(), bz.BZ_FP64, idx.data_ptr(), c1, 0, got.data_ptr(),
                                    bz.BZ_SCATTER, stream)
        torch.cuda.synchronize()
        assert torch.equal(got, ref)
        # call 2, smaller: the first c2 rows, compact output
        ref2 = col(f[:c2])
        got2 = torch.empty_like(ref2)
        bz.bz_collide_batch_noalloc(p, f.data_ptr(), bz.BZ_FP64, 0, c2, 0, got2.data_ptr(), 0, stream)
        torch.cuda.synchronize()
        assert torch.equal(got2, ref2)
        assert torch.isfinite(got2).all()
    finally:
        col.close()
        bz.bz_plan_destroy(p)
