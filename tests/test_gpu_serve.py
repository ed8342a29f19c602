"""GPU tests of the serving runtime (bz_server_* / bz_serve_*): requests from
several client threads with different grid sizes and cell counts; results are
bitwise equal to a direct bz_collide_batch of the same operator, a request's
result is the same alone and in the mix, and a sampled cell of every served
request matches the FP64 oracle (per-cell error <= 1e-5 with the
near-equilibrium floor, FP32 plans; moment drift <= 1e-12 after the FP64
projection); admission never exceeds the arena, and a request that fits the
arena only after its own plan's tables move is still admitted; failed
requests do not disturb the others; a request waits for the caller's
pending writes of its input."""
import threading
import time

import numpy as np
import pytest

import bz_inputs as gen
from oracle import spectral
from tests.gpu_util import oracle_plan

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def plan(bz, n, m=8, precision=1):
    return bz.make_plan_desc(n=n, L=8.0, m=m, dir_kind=bz.BZ_DIRS_SPIRAL, precision=precision)


def wait(srv, ticket, timeout=60.0):
    t0 = time.time()
    while True:
        done, res = srv.poll(ticket)
        if done:
            return res
        assert time.time() - t0 < timeout, "request did not finish"
        time.sleep(0.0005)


def inputs(n, cells, seed):
    return torch.from_numpy(gen.bimaxwellian_batch(cells, n, 8.0, seed=seed)).cuda()


class OracleCells:
    """FP64 oracle of the m = 8 spiral operator the serving tests request,
    memoised per (input key, cell)."""

    def __init__(self):
        self.plans, self.memo = {}, {}

    def check(self, key, f, q, cell, tol=1e-5):
        n = f.shape[-1]
        if n not in self.plans:
            self.plans[n] = oracle_plan(n, rule="spiral", m=8)
        if (key, cell) not in self.memo:
            fc = f[cell].double().cpu().numpy()
            qq, _, ql = spectral.collide_parts(fc, self.plans[n])
            self.memo[(key, cell)] = (spectral.project(qq, n, 8.0), ql)
        ref, loss = self.memo[(key, cell)]
        got = q[cell].cpu().numpy()
        err = spectral.rel_err(got, ref, loss)
        assert err <= tol, (key, cell, err)
        assert spectral.moment_drift(got, n, 8.0) <= 1e-12


def test_serve_matches_direct_and_mix():
    import paper_2505_03360_amd as bz
    print("case serve mix", flush=True)
    srv = bz.Server(arena_bytes=2 << 30, max_inflight=6, n_streams=3)
    work = [(16, 5, 1), (24, 3, 2), (32, 4, 3), (16, 37, 4), (32, 9, 5), (24, 11, 6)]
    fs = {k: inputs(n, c, s) for k, (n, c, s) in enumerate(work)}
    orc = OracleCells()
    # alone: one request at a time
    alone = {}
    for k, (n, c, s) in enumerate(work):
        q = torch.empty((c, n, n, n), dtype=torch.float64, device="cuda")
        res = wait(srv, srv.submit(fs[k], q, plan(bz, n)))
        assert res.state == bz.BZ_REQ_DONE and res.err == 0
        assert res.t_submit_ns <= res.t_admit_ns <= res.t_done_ns
        alone[k] = q.clone()
        orc.check(k, fs[k], q, (3 * k) % c)
    # in the mix: all requests from three client threads at once, twice each
    outs = {}

    def client(keys):
        tickets = []
        for k in keys:
            n, c, _ = work[k]
            for r in range(2):
                q = torch.empty((c, n, n, n), dtype=torch.float64, device="cuda")
                outs[(k, r)] = q
                tickets.append(srv.submit(fs[k], q, plan(bz, n), client_id=k))
        for t in tickets:
            res = wait(srv, t)
            assert res.state == bz.BZ_REQ_DONE, res.err
    th = [threading.Thread(target=client, args=(ks,)) for ks in ([0, 3], [1, 4], [2, 5])]
    for t in th:
        t.start()
    for t in th:
        t.join()
    torch.cuda.synchronize()
    for (k, r), q in outs.items():
        assert torch.equal(q, alone[k]), (k, r)
        orc.check(k, fs[k], q, (5 * k + 2 * r + 1) % work[k][1])
    # and equal to a direct call of the same operator
    for k, (n, c, s) in enumerate(work):
        col = bz.Collider(n, c, L=8.0, m=8, dir_kind=bz.BZ_DIRS_SPIRAL, precision=1)
        assert torch.equal(col(fs[k]), alone[k])
    st = srv.stats()
    assert st.completed == 18 and st.failed == 0 and st.p99_ms >= st.p50_ms > 0
    assert bz.bz_server_stats(srv.handle) == (st.p50_ms, st.p99_ms, st.cells_per_s)
    srv.close()


def test_admission_bounded_by_arena():
    import paper_2505_03360_amd as bz
    print("case serve arena", flush=True)
    n, cells = 32, 16
    pd = plan(bz, n)
    p = bz.bz_plan_create(bz.make_plan_desc(n=n, L=8.0, m=8, dir_kind=bz.BZ_DIRS_SPIRAL, precision=1))
    tb, fixed, per = bz.bz_plan_device_bytes(p)
    bz.bz_plan_destroy(p)
    arena = tb + 2 * (fixed + per * cells) + 4096  # tables + two requests
    srv = bz.Server(arena_bytes=arena, max_inflight=8, n_streams=4)
    f = inputs(n, cells, 7)
    qs = [torch.empty((cells, n, n, n), dtype=torch.float64, device="cuda") for _ in range(10)]
    ts = [srv.submit(f, q, pd) for q in qs]
    for t in ts:
        assert wait(srv, t).state == bz.BZ_REQ_DONE
    st = srv.stats()
    assert st.arena_peak <= arena
    for q in qs[1:]:
        assert torch.equal(q, qs[0])
    srv.close()


def test_failed_requests_are_isolated():
    import paper_2505_03360_amd as bz
    print("case serve failures", flush=True)
    # an arena of 48 MB: one 2048-cell slice of an N = 16 request needs ~100 MB of workspace
    srv = bz.Server(arena_bytes=48 << 20, max_inflight=4, n_streams=2)
    f = inputs(16, 4, 8)
    good = torch.empty((4, 16, 16, 16), dtype=torch.float64, device="cuda")
    bad_n = bz.make_plan_desc(n=20, L=8.0, m=8, dir_kind=bz.BZ_DIRS_SPIRAL)
    t_bad = srv.submit(f, good, bad_n)
    big_f = torch.zeros((4096, 16, 16, 16), dtype=torch.float64, device="cuda")  # valid buffers, never read
    big_q = torch.empty_like(big_f)
    t_huge = srv.submit(big_f, big_q, plan(bz, 16))  # its slice can never fit the arena
    t_good = srv.submit(f, good, plan(bz, 16))
    r_bad, r_huge, r_good = wait(srv, t_bad), wait(srv, t_huge), wait(srv, t_good)
    assert r_bad.state == bz.BZ_REQ_FAILED and r_bad.err == bz.BZ_ERR_UNSUPPORTED
    assert r_huge.state == bz.BZ_REQ_FAILED and r_huge.err == bz.BZ_ERR_NOMEM
    assert r_good.state == bz.BZ_REQ_DONE
    with pytest.raises(bz.BzError):
        srv.poll(t_good)  # already collected
    with pytest.raises(ValueError):  # buffers smaller than the cells named: refused by the binding
        srv.submit(f, good, plan(bz, 16), ncells=400000)
    st = srv.stats()
    assert st.failed == 2 and st.completed == 1
    srv.close()


def test_nonfinite_output_fails_only_its_request():
    import paper_2505_03360_amd as bz
    print("case serve nonfinite", flush=True)
    srv = bz.Server(arena_bytes=1 << 30, max_inflight=4, n_streams=2)
    good = inputs(16, 3, 21)
    bad = inputs(16, 3, 22)
    bad[1, 5, 6, 7] = float("nan")
    qg = torch.empty((3, 16, 16, 16), dtype=torch.float64, device="cuda")
    qb = torch.empty_like(qg)
    tb = srv.submit(bad, qb, plan(bz, 16))
    tg = srv.submit(good, qg, plan(bz, 16))
    rb, rg = wait(srv, tb), wait(srv, tg)
    assert rb.state == bz.BZ_REQ_FAILED and rb.err == bz.BZ_ERR_NUMERIC
    assert rg.state == bz.BZ_REQ_DONE and rg.err == 0
    # the next request on the same cached plan and arena starts clean
    t2 = srv.submit(good, qg, plan(bz, 16))
    r2 = wait(srv, t2)
    assert r2.state == bz.BZ_REQ_DONE and r2.err == 0
    srv.close()


def test_admission_moves_the_plans_own_tables():
    """With nothing in flight, a request whose workspace fits the arena only
    once its own plan's tables are moved (they split the free space) is
    admitted: the tables are dropped, the workspace placed, the tables
    uploaded again after it.  The request sequence builds that layout: plan
    P1's tables at the front, then P2's, P1 evicted, and a large P2 request."""
    import paper_2505_03360_amd as bz
    print("case serve fragmented arena", flush=True)
    n = 16
    p1 = bz.make_plan_desc(n=n, L=8.0, m=8, dir_kind=bz.BZ_DIRS_SPIRAL, precision=1)
    p2 = bz.make_plan_desc(n=n, L=8.0, m=6, dir_kind=bz.BZ_DIRS_ICOSA6, precision=1)

    def sizes(pd, cells):
        d = bz.make_plan_desc(n=n, L=8.0, m=pd.m, dir_kind=pd.dir_kind, precision=1, max_cells=cells)
        h = bz.bz_plan_create(d)
        tb, fixed, per = bz.bz_plan_device_bytes(h)
        bz.bz_plan_destroy(h)
        a = lambda x: (x + 255) // 256 * 256
        return a(tb), lambda c: a(fixed + per * c)
    t1, ws1 = sizes(p1, 1)
    t2, ws2 = sizes(p2, 1)  # requests up to 256 cells share one plan (one chunk class)
    c3 = 1
    while ws2(c3) <= t1 + 4096:  # the large request's workspace exceeds P1's tables
        c3 *= 2
    assert c3 <= 256
    arena = t2 + ws2(c3) + 256  # fits only as [workspace | P2 tables]
    assert t1 + t2 + ws2(1) <= arena and ws2(c3) > arena - t1 - t2
    srv = bz.Server(arena_bytes=arena, max_inflight=1, n_streams=1)
    f = inputs(n, c3, 31)
    q1 = torch.empty((1, n, n, n), dtype=torch.float64, device="cuda")
    assert wait(srv, srv.submit(f[:1], q1, p1)).state == bz.BZ_REQ_DONE
    q2 = torch.empty((1, n, n, n), dtype=torch.float64, device="cuda")
    assert wait(srv, srv.submit(f[:1], q2, p2)).state == bz.BZ_REQ_DONE
    q3 = torch.empty((c3, n, n, n), dtype=torch.float64, device="cuda")
    r3 = wait(srv, srv.submit(f, q3, p2), timeout=60.0)
    assert r3.state == bz.BZ_REQ_DONE and r3.err == 0
    assert torch.equal(q3[:1], q2)
    st = srv.stats()
    assert st.arena_peak <= arena and st.completed == 3
    srv.close()


def test_request_waits_for_pending_input_writes():
    """The input is produced by a long queue of kernels on the caller's stream
    right before submission; the served result equals the one computed after a
    full synchronisation."""
    import paper_2505_03360_amd as bz
    print("case serve ready event", flush=True)
    n, c = 32, 64
    src = inputs(n, c, 41)
    f = torch.zeros_like(src)
    srv = bz.Server(arena_bytes=1 << 30, max_inflight=2, n_streams=2)
    pd = plan(bz, n)
    q_ref = torch.empty((c, n, n, n), dtype=torch.float64, device="cuda")
    torch.cuda.synchronize()
    for _ in range(50):  # a long chain of dependent writes ending in f == src
        f.mul_(0.5).add_(src, alpha=0.5)
    f.copy_(src)
    q = torch.empty_like(q_ref)
    t = srv.submit(f, q, pd)
    assert wait(srv, t).state == bz.BZ_REQ_DONE
    torch.cuda.synchronize()
    assert wait(srv, srv.submit(src, q_ref, pd)).state == bz.BZ_REQ_DONE
    assert torch.equal(q, q_ref)
    srv.close()


def test_sliced_requests_match_direct_slices():
    """With slice_cells = 16, requests of 40 cells run as slices of 16, 16 and
    8 cells (one at a time, on the least loaded stream): the result equals a
    direct bz_collide_batch of each slice with a plan of that size, compact
    and scattered, alone and beside other requests; one cell against the
    oracle."""
    import paper_2505_03360_amd as bz
    print("case serve sliced", flush=True)
    n, c = 16, 40
    srv = bz.Server(arena_bytes=1 << 30, max_inflight=6, n_streams=3, slice_cells=16)
    f = inputs(n, 2 * c, 51)
    col = bz.Collider(n, 16, L=8.0, m=8, dir_kind=bz.BZ_DIRS_SPIRAL, precision=1)
    direct = torch.cat([col(f[a:b]) for a, b in ((0, 16), (16, 32), (32, 40))])
    idx = torch.arange(2 * c - 1, 0, -2, dtype=torch.int32, device="cuda")  # rows 79, 77, ..., 1
    dsc = torch.zeros((2 * c, n, n, n), dtype=torch.float64, device="cuda")
    for a, b in ((0, 16), (16, 32), (32, 40)):
        col(f, idx=idx[a:b].contiguous(), out=dsc, scatter=True)
    q = torch.empty((c, n, n, n), dtype=torch.float64, device="cuda")
    assert wait(srv, srv.submit(f[:c], q, plan(bz, n))).state == bz.BZ_REQ_DONE
    assert torch.equal(q, direct)
    qs = torch.zeros_like(dsc)
    assert wait(srv, srv.submit(f, qs, plan(bz, n), idx=idx, scatter=True)).state == bz.BZ_REQ_DONE
    assert torch.equal(qs, dsc)
    # in a mix with small requests of other sizes
    small = inputs(24, 5, 52)
    outs = []
    tickets = []
    for r in range(3):
        qq = torch.empty_like(q)
        qsm = torch.empty((5, 24, 24, 24), dtype=torch.float64, device="cuda")
        tickets.append(srv.submit(f[:c], qq, plan(bz, n), client_id=r))
        tickets.append(srv.submit(small, qsm, plan(bz, 24), client_id=r))
        outs.append(qq)
    for t in tickets:
        assert wait(srv, t).state == bz.BZ_REQ_DONE
    for qq in outs:
        assert torch.equal(qq, direct)
    OracleCells().check("sliced", f[:c], q, 37)
    srv.close()


def test_admission_prefers_short_requests_with_bounded_bypass():
    """One in-flight slot.  While a long request runs, a second long request
    and then twelve short ones queue: admission takes the least work first, so
    short requests pass the queued long one, but at most nine of them (a
    request passed over more than eight times goes first).  Every result
    equals the same request served alone."""
    import paper_2505_03360_amd as bz
    print("case serve admission order", flush=True)
    n, big, small = 48, 2048, 16
    pd = plan(bz, n)
    srv = bz.Server(arena_bytes=16 << 30, max_inflight=1, n_streams=1)
    f = inputs(n, 64, 61).repeat(big // 64, 1, 1, 1).contiguous()
    ref = {}
    for c in (big, small):  # builds both plans (request sizes map to plan classes)
        ref[c] = torch.empty((c, n, n, n), dtype=torch.float64, device="cuda")
        assert wait(srv, srv.submit(f[:c], ref[c], pd)).state == bz.BZ_REQ_DONE
    qa, qb = (torch.empty((big, n, n, n), dtype=torch.float64, device="cuda") for _ in range(2))
    qs = [torch.empty((small, n, n, n), dtype=torch.float64, device="cuda") for _ in range(12)]
    ta = srv.submit(f, qa, pd)
    tb = srv.submit(f, qb, pd)
    ts = [srv.submit(f[:small], q, pd) for q in qs]
    ra, rb = wait(srv, ta), wait(srv, tb)
    rs = [wait(srv, t) for t in ts]
    assert all(r.state == bz.BZ_REQ_DONE for r in [ra, rb] + rs)
    before_b = sum(r.t_admit_ns < rb.t_admit_ns for r in rs)
    assert 1 <= before_b <= 9, before_b
    assert torch.equal(qa, ref[big]) and torch.equal(qb, ref[big])
    for q in qs:
        assert torch.equal(q, ref[small])
    srv.close()
