"""Host-side serving logic (CPU only): request checks, footprint bounds,
budget admission, rejection paths."""
import types

import numpy as np

import spgen
from paper_2106_14402_amd import serve as SV


def fake_graph(n=1000, seed=0):
    rng = np.random.default_rng(seed)
    A = spgen.rmat_graph(0, 6, rng, symmetric=False, n=n)
    g = types.SimpleNamespace(n=n, outdeg=np.diff(A.ptr).astype(np.int64), device=None)
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
    budget = sum(sorted(bounds)[:2]) + 1
    srv = SV.FrontierServer(g, hbm_budget=budget, workers=1)
    for i, F in enumerate(reqs):
        if bounds[i] <= budget:
            assert srv.submit(i, F, 0.0) is None
    srv._feeding = False
    taken = 0
    while srv._pending:
        batch, need = srv._take_batch()
        assert need <= budget
        assert srv._in_flight <= budget
        taken += len(batch)
        srv._release(need)
    assert taken == sum(1 for b in bounds if b <= budget)
    # a request larger than the whole budget is rejected with SPG_E_NOMEM
    big = max(range(len(reqs)), key=lambda i: bounds[i])
    srv2 = SV.FrontierServer(g, hbm_budget=bounds[big] - 1, workers=1)
    r = srv2.submit(99, reqs[big], 0.0)
    assert r is not None and r.status == SV.SPG_E_NOMEM
    # an invalid frontier is rejected with SPG_E_INVALID and queues nothing
    bad = spgen.SparseMatrix(1, g.n, "csr", np.array([0, 1]), np.array([g.n + 5], np.int32), None)
    r = srv2.submit(100, bad, 0.0)
    assert r is not None and r.status == SV.SPG_E_INVALID
    assert not srv2._pending


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
