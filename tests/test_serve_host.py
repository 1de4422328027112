"""Host-side serving logic (CPU only): request checks, footprint bounds,
budget admission, rejection paths."""
import types

import numpy as np

import spgen
from paper_2106_14402_amd import serve as SV


def fake_graph(n=1000, seed=0):
    """Host stand-in of a ResidentGraph: degrees for the bounds, and a
    descriptor whose device addresses are never dereferenced (plan creation
    and workspace sizing are host-only)."""
    from paper_2106_14402_amd import binding as B
    rng = np.random.default_rng(seed)
    A = spgen.rmat_graph(0, 6, rng, symmetric=False, n=n)
    desc = B.spg_matrix(n, n, A.nnz, B.SPG_CSR, 0x10000, 0x20000, None)
    g = types.SimpleNamespace(n=n, outdeg=np.diff(A.ptr).astype(np.int64), device=None,
                              A=types.SimpleNamespace(descriptor=lambda: desc))
    return g, A


def test_check_frontier():
    g, _ = fake_graph()
    rng = np.random.default_rng(1)
    Ft = spgen.frontier(g.n, 5, rng)
    assert SV.check_frontier(g, Ft)
    bad = Ft.with_values(None)
    bad.idx = Ft.idx.copy()
    bad.idx[0] = g.n                                         # out of range
    assert not SV.check_frontier(g, bad)
    uns = spgen.SparseMatrix(1, g.n, "csr", np.array([0, 2]), np.array([5, 3], np.int32), None)
    assert not SV.check_frontier(g, uns)                     # unsorted sources
    dup = spgen.SparseMatrix(1, g.n, "csr", np.array([0, 2]), np.array([3, 3], np.int32), None)
    assert not SV.check_frontier(g, dup)                     # duplicate source
    wrong = spgen.SparseMatrix(1, g.n + 1, "csr", np.array([0, 1]), np.array([3], np.int32), None)
    assert not SV.check_frontier(g, wrong)


def test_bound_covers_output():
    g, A = fake_graph()
    rng = np.random.default_rng(2)
    for _ in range(20):
        Ft = spgen.frontier(g.n, int(rng.integers(1, 40)), rng)
        # exact output size: union of out-neighbour lists per row
        out = 0
        for r in range(Ft.nrows):
            s = set()
            for v in Ft.idx[Ft.ptr[r]:Ft.ptr[r + 1]]:
                s |= set(A.idx[A.ptr[v]:A.ptr[v + 1]].tolist())
            out += len(s)
        assert SV.request_bound_bytes(g, Ft) >= 4 * out + 8 * (Ft.nrows + 1)


def test_admission_respects_budget_and_rejects():
    g, _ = fake_graph()
    rng = np.random.default_rng(3)
    reqs = [spgen.frontier(g.n, 3, rng) for _ in range(6)]
    bounds = [SV.request_bound_bytes(g, F) for F in reqs]
    probe = SV.FrontierServer(g, workers=1)
    alone = [b + probe.workspace_bytes(F.nrows, F.nnz) for b, F in zip(bounds, reqs)]
    budget = sum(sorted(alone)[:2]) + 1
    srv = SV.FrontierServer(g, hbm_budget=budget, workers=1)
    for i, F in enumerate(reqs):
        if alone[i] <= budget:
            assert srv.submit(i, F, 0.0) is None
    srv._feeding = False
    taken = 0
    while srv._pending:
        batch, need = srv._take_batch()
        rows = sum(F.nrows for _, _, F, _ in batch)
        ents = sum(F.nnz for _, _, F, _ in batch)
        # admitted bytes: the requests' bounds plus their product's workspace
        assert need == sum(b for _, _, _, b in batch) + srv.workspace_bytes(rows, ents)
        assert need <= budget
        assert srv._in_flight <= budget
        taken += len(batch)
        srv._release(need)
    assert taken == sum(1 for a in alone if a <= budget)
    # a request larger than the whole budget is rejected with SPG_E_NOMEM
    big = max(range(len(reqs)), key=lambda i: alone[i])
    srv2 = SV.FrontierServer(g, hbm_budget=alone[big] - 1, workers=1)
    r = srv2.submit(99, reqs[big], 0.0)
    assert r is not None and r.status == SV.SPG_E_NOMEM
    # an invalid frontier is rejected with SPG_E_INVALID and queues nothing
    bad = spgen.SparseMatrix(1, g.n, "csr", np.array([0, 1]), np.array([g.n + 5], np.int32), None)
    r = srv2.submit(100, bad, 0.0)
    assert r is not None and r.status == SV.SPG_E_INVALID
    assert not srv2._pending


def test_admission_counts_the_workspace():
    """The workspace the plan asks for (offsets, row lists, panel indexes of
    the resident operand, sort room for the frontier) is part of a request's
    admitted bytes: a budget that covers the bound alone rejects it."""
    g, _ = fake_graph()
    F = spgen.frontier(g.n, 8, np.random.default_rng(5))
    bound = SV.request_bound_bytes(g, F)
    srv = SV.FrontierServer(g, workers=1)
    ws = srv.workspace_bytes(F.nrows, F.nnz)
    assert ws > 0
    tight = SV.FrontierServer(g, hbm_budget=bound + ws - 1, workers=1)
    r = tight.submit(1, F, 0.0)
    assert r is not None and r.status == SV.SPG_E_NOMEM
    ok = SV.FrontierServer(g, hbm_budget=bound + ws, workers=1)
    assert ok.submit(1, F, 0.0) is None


def test_worker_survives_a_failing_batch():
    """An exception that is not an SpgError (a torch allocation failure, say)
    turns the batch's requests into error results; the worker keeps going and
    the budget is released."""
    import threading
    g, _ = fake_graph()
    rng = np.random.default_rng(6)
    srv = SV.FrontierServer(g, workers=1)
    calls = []

    def failing(batch, stream):
        calls.append(len(batch))
        if len(calls) == 1:
            raise RuntimeError("out of memory")
        return [SV.Result(rid, SV.SPG_OK, arr) for arr, rid, _, _ in batch]

    srv._execute = failing
    srv._feeding = True
    for i in range(3):
        srv.submit(i, spgen.frontier(g.n, 2, rng), 0.0)
    t = threading.Thread(target=srv._worker_loop, args=(None,), daemon=True)
    t.start()
    import time

    def wait_for(n):
        t_end = time.time() + 10
        while len(srv._results) < n and t.is_alive() and time.time() < t_end:
            time.sleep(0.01)

    wait_for(3)                          # the first batch failed
    for i in range(3, 5):
        srv.submit(i, spgen.frontier(g.n, 2, rng), 0.0)
    wait_for(5)
    with srv._cv:
        srv._feeding = False
        srv._stop = True
        srv._cv.notify_all()
    t.join(timeout=10)
    assert not t.is_alive()
    st = {r.rid: r.status for r in srv._results}
    assert all(st[i] == SV.SPG_E_DEVICE for i in range(3))
    assert all(st[i] == SV.SPG_OK for i in range(3, 5))
    assert srv._in_flight == 0


def test_batch_caps():
    g, _ = fake_graph()
    rng = np.random.default_rng(4)
    srv = SV.FrontierServer(g, hbm_budget=1 << 40, max_batch_rows=10, max_batch_requests=3, workers=1)
    for i in range(8):
        srv.submit(i, spgen.frontier(g.n, 4, rng), 0.0)
    batch, need = srv._take_batch()
    assert len(batch) == 2                  # 4 + 4 rows; a third would exceed 10
    srv._release(need)
    srv.max_rows = 1000
    batch, need = srv._take_batch()
    assert len(batch) == 3                  # request cap


def test_cancel_withdraws_a_waiting_request():
    """cancel() removes a request no worker has taken: it completes with
    status CANCELLED and is never admitted; the others are taken as before."""
    g, _ = fake_graph()
    rng = np.random.default_rng(4)
    reqs = [spgen.frontier(g.n, 3, rng) for _ in range(4)]
    srv = SV.FrontierServer(g, workers=1)
    for i, F in enumerate(reqs):
        assert srv.submit(i, F, 0.0) is None
    assert srv.cancel(2)
    assert not srv.cancel(2)      # no longer waiting
    assert not srv.cancel(99)     # unknown
    srv._feeding = False
    taken = []
    while srv._pending:
        batch, need = srv._take_batch()
        taken += [rid for _, rid, _, _ in batch]
        srv._release(need)
    assert sorted(taken) == [0, 1, 3]
    assert [(r.rid, r.status) for r in srv._results] == [(2, SV.CANCELLED)]
    assert srv._in_flight == 0


def test_deadline_expires_waiting_requests_only():
    """A request whose deadline passes while it waits completes with status
    EXPIRED; one taken before its deadline is not touched; a request with
    no deadline waits as long as it must."""
    import time
    g, _ = fake_graph()
    rng = np.random.default_rng(5)
    reqs = [spgen.frontier(g.n, 3, rng) for _ in range(3)]
    srv = SV.FrontierServer(g, workers=1, max_batch_requests=1)
    now = time.perf_counter()
    assert srv.submit(0, reqs[0], now, deadline=now + 60.0) is None   # taken in time
    assert srv.submit(1, reqs[1], now, deadline=now - 1.0) is None    # already past
    assert srv.submit(2, reqs[2], now) is None                        # no deadline
    srv._feeding = False
    taken = []
    while srv._pending:
        batch, need = srv._take_batch()
        if batch is None:
            break
        taken += [rid for _, rid, _, _ in batch]
        srv._release(need)
    assert taken == [0, 2]
    assert [(r.rid, r.status) for r in srv._results] == [(1, SV.EXPIRED)]
    assert not srv._deadline
