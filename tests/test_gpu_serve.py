"""Served frontier expansion on the GPU: each result equals the same request
computed alone and the union of out-neighbour lists of its sources; tight
HBM budgets queue requests; bad requests are rejected without affecting the
others."""
import numpy as np
import pytest

import spgen

pytestmark = pytest.mark.gpu


def _graph(scale=14, seed=41):
    return spgen.rmat_graph(scale, 16, np.random.default_rng(seed), symmetric=False)


def _union_rows(A, Ft):
    rows = []
    for r in range(Ft.nrows):
        src = Ft.idx[Ft.ptr[r]:Ft.ptr[r + 1]]
        parts = [A.idx[A.ptr[v]:A.ptr[v + 1]] for v in src]
        rows.append(np.unique(np.concatenate(parts)) if parts else np.zeros(0, np.int32))
    return rows


def _check(res, A, Ft, alone):
    assert res.status == 0
    ap, ai = alone
    assert np.array_equal(res.ptr, ap) and np.array_equal(res.idx, ai), "differs from alone"
    want = _union_rows(A, Ft)
    for r, w in enumerate(want):
        assert np.array_equal(res.idx[res.ptr[r]:res.ptr[r + 1]], w)


def test_served_equals_alone_and_union():
    from paper_2106_14402_amd import serve as SV
    A = _graph()
    g = SV.ResidentGraph(A)
    reqs = spgen.request_stream(A.nrows, 150, rate=20000.0, rng=np.random.default_rng(5), k_max=64)
    srv = SV.FrontierServer(g, hbm_budget=1 << 30, workers=3)
    results = srv.serve(reqs)
    assert len(results) == len(reqs)
    assert max(r.batch_rows for r in results) > max(q.k for q in reqs)  # batching happened
    for q, r in zip(reqs, results):
        _check(r, A, q.Ft, SV.expand_alone(g, q.Ft))


def test_large_output_rows_use_dense_panels():
    """Sources with the largest out-degrees: rows beyond the hash classes."""
    from paper_2106_14402_amd import serve as SV
    A = _graph(scale=17, seed=42)
    g = SV.ResidentGraph(A)
    deg = np.diff(A.ptr)
    hubs = np.argsort(deg)[::-1][:64]
    rows = [np.sort(hubs[:64]), np.sort(hubs[10:30]), np.sort(hubs[:3])]
    ptr = np.cumsum([0] + [len(x) for x in rows])
    Ft = spgen.SparseMatrix(len(rows), A.nrows, "csr", ptr.astype(np.int64),
                            np.concatenate(rows).astype(np.int32), None)
    from paper_2106_14402_amd import binding
    # narrow symbolic panels so several panels (and the cached index) are used
    o = binding.make_options(sym_panel_log2=14)
    srv = SV.FrontierServer(g, hbm_budget=1 << 32, workers=1, options=o)
    req = [type("R", (), {"rid": 0, "arrival": 0.0, "Ft": Ft})()]
    res = srv.serve(req)[0]
    _check(res, A, Ft, SV.expand_alone(g, Ft, o))


def test_tight_budget_queues_and_rejects():
    """A request is rejected when its own bound plus the workspace of a batch
    holding it alone exceeds the budget; the others queue and complete."""
    from paper_2106_14402_amd import serve as SV
    A = _graph()
    g = SV.ResidentGraph(A)
    reqs = spgen.request_stream(A.nrows, 60, rate=50000.0, rng=np.random.default_rng(6), k_max=16)
    bounds = [SV.request_bound_bytes(g, q.Ft) + g.workspace_bytes(q.Ft.nrows, q.Ft.nnz) for q in reqs]
    budget = int(np.percentile(bounds, 60)) + int(np.percentile(bounds, 10))
    assert 0 < sum(b > budget for b in bounds) < len(bounds)
    bad = spgen.SparseMatrix(1, A.nrows, "csr", np.array([0, 1]), np.array([A.nrows + 3], np.int32), None)
    reqs.append(type("R", (), {"rid": 1000, "arrival": reqs[-1].arrival, "Ft": bad})())
    srv = SV.FrontierServer(g, hbm_budget=budget, workers=2)
    results = srv.serve(reqs)
    by = {r.rid: r for r in results}
    assert by[1000].status == SV.SPG_E_INVALID
    for q, b in zip(reqs[:-1], bounds):
        r = by[q.rid]
        if b > budget:
            assert r.status == SV.SPG_E_NOMEM
        else:
            _check(r, A, q.Ft, SV.expand_alone(g, q.Ft))


def test_deadlines_under_overload():
    """Requests offered far above the service rate with a short wait limit:
    every request has exactly one result, each either completed (and equal
    to its product alone) or expired while waiting; with no limit all
    complete."""
    from paper_2106_14402_amd import serve as SV
    A = _graph()
    g = SV.ResidentGraph(A)
    reqs = spgen.request_stream(A.nrows, 120, rate=1e6, rng=np.random.default_rng(8), k_max=64)
    srv = SV.FrontierServer(g, workers=1, max_batch_requests=4)
    results = srv.serve(reqs, timeout_s=0.002)
    assert sorted(r.rid for r in results) == sorted(q.rid for q in reqs)
    by = {r.rid: r for r in results}
    done = [q for q in reqs if by[q.rid].status == SV.SPG_OK]
    assert all(by[q.rid].status in (SV.SPG_OK, SV.EXPIRED) for q in reqs)
    assert done
    for q in done[:20]:
        _check(by[q.rid], A, q.Ft, SV.expand_alone(g, q.Ft))
    again = SV.FrontierServer(g, workers=1, max_batch_requests=4).serve(reqs)
    assert all(r.status == SV.SPG_OK for r in again)
