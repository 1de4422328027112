"""Parity at the full workload sizes, in the launch configurations that
bench.py times.

The outputs are too large for the oracle to hand over whole (R-MAT scale 20
squared has 2.4e10 entries).  For the R-MAT square every output slice is
compared through digests: the oracle formed every slice once, hashed it and
stored the digests of blocks of 1024 slices (tests/golden), and the device
result is hashed the same way here.  Each test also compares a seeded sample
of output slices with the oracle computed for exactly those slices (its
row/column selection), and checks properties that hold at any size over the
whole output on the device: every slice sorted strictly ascending, ids in
range, the two R-MAT semirings giving one pattern, value bounds, column sums
of a column-stochastic square, prune counts.
"""
import os

import numpy as np
import pytest

import oracle
import spgen
from tests.gpu_util import assert_parity

pytestmark = [pytest.mark.gpu, pytest.mark.slow]

NTHREADS = min(16, os.cpu_count() or 1)


def _sample(weights, rng, n_top=1, n_heavy=8, n_rand=48):
    """Sorted, distinct slice ids: the heaviest, a few from the top 1% and
    uniform ones, plus the first and last slice (ragged ends)."""
    n = weights.size
    order = np.argsort(weights, kind="stable")[::-1]
    top1 = order[:max(1, n // 100)]
    pick = [order[:n_top], rng.choice(top1, size=min(n_heavy, top1.size), replace=False),
            rng.choice(n, size=n_rand, replace=False), [0, n - 1]]
    return np.unique(np.concatenate([np.asarray(p, np.int64) for p in pick]))


def _fetch(C, rows, with_val=True):
    """Pack the given slices of a device result on the host."""
    import torch
    ptr = C.ptr.cpu().numpy()
    nptr = np.zeros(rows.size + 1, np.int64)
    idx, val = [], []
    for i, r in enumerate(rows):
        lo, hi = int(ptr[r]), int(ptr[r + 1])
        nptr[i + 1] = nptr[i] + hi - lo
        idx.append(C.idx[lo:hi].cpu().numpy())
        if with_val and C.val is not None:
            val.append(C.val[lo:hi].cpu().numpy())
    torch.cuda.synchronize()
    gi = np.concatenate(idx) if idx else np.zeros(0, np.int32)
    gv = np.concatenate(val) if val else None
    return nptr, gi, gv


def _check_sorted_in_range(C, nminor, chunk=1 << 30):
    """Every slice strictly ascending and every id in [0, nminor), over the
    whole device output, a chunk at a time."""
    import torch
    nnz = int(C.idx.numel())
    if nnz == 0:
        return
    ptr = C.ptr
    for lo in range(0, nnz, chunk):
        hi = min(nnz, lo + chunk + 1)
        x = C.idx[lo:hi]
        assert int(x.min()) >= 0 and int(x.max()) < nminor
        bad = torch.nonzero(x[1:] <= x[:-1]).flatten() + (lo + 1)   # positions that do not ascend
        if bad.numel():
            # each must start a slice: it appears in ptr
            pos = torch.searchsorted(ptr, bad)
            ok = (pos < ptr.numel()) & (ptr[pos.clamp(max=ptr.numel() - 1)] == bad)
            assert bool(ok.all()), "an output slice is not strictly ascending"


# --------------------------------------------------------------------------
# R-MAT scale 20 squared: (OR,AND) pattern and (min,+) int32
# --------------------------------------------------------------------------
@pytest.fixture(scope="module")
def rmat20():
    A = spgen.config_rmat()
    return A, oracle.flops(A, A)


GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "rmat20_digests.json")


def _golden(sr):
    """Block digests of the whole R-MAT scale-20 square written by the
    oracle (tests/golden/make_rmat20_digests.py), or None if absent."""
    import json
    if not os.path.exists(GOLDEN):
        return None
    with open(GOLDEN) as f:
        rec = json.load(f)
    g = rec["semirings"].get(sr)
    if g is None:
        return None
    bh = np.array([int(x, 16) for x in g["block_hash"]], dtype=np.uint64)
    return rec["block"], np.asarray(g["block_nnz"], np.int64), bh


def _check_every_row(C, M, sr, nrows):
    """Every output slice against the oracle: block digests of the device
    result equal the oracle's; on a mismatch the first differing slice is
    found and compared with the oracle's own computation of it."""
    from tests import digest_util as D
    g = _golden(sr)
    if g is None:
        return False
    block, want_n, want_h = g
    got_n, got_h = D.block_digests(C.ptr, C.idx, C.val, nrows, block=block)
    assert got_n.size == want_n.size
    bad = np.nonzero((got_n != want_n) | (got_h != want_h))[0]
    if bad.size:
        b = int(bad[0])
        rows = np.arange(b * block, min(nrows, (b + 1) * block))
        n, h = D.slice_digests(C.ptr, C.idx, C.val, int(rows[0]), int(rows[-1]) + 1)
        on, oh = oracle.digest(M, M, sr, select=rows, nthreads=NTHREADS)
        diff = np.nonzero((n.cpu().numpy() != on) | (h.cpu().numpy().view(np.uint64) != oh))[0]
        r = int(rows[diff[0]]) if diff.size else -1
        detail = ""
        if r >= 0:
            want = oracle.spgemm(M, M, sr, select=[r], nthreads=NTHREADS)
            got = _fetch(C, np.array([r]))
            detail = (f"; slice {r}: {got[1].size} entries on the device, {want[1].size} in the oracle, "
                      f"ids equal: {np.array_equal(got[1], want[1])}")
        raise AssertionError(f"{bad.size} of {want_n.size} blocks differ (first block {b}){detail}")
    return True


def test_rmat20_bool_and_min_plus(rmat20):
    import torch

    from paper_2106_14402_amd import binding as B
    from paper_2106_14402_amd import spgemm as S
    A, fl = rmat20
    rows = _sample(fl, np.random.default_rng(11))
    print(f"[fullsize] R-MAT s20 sample of {rows.size} rows, {int(fl[rows].sum())} flops", flush=True)
    dA = S.to_device(A)
    Apat = S.DeviceMatrix(dA.nrows, dA.ncols, "csr", dA.ptr, dA.idx, None)
    Hpat = A.with_values(None)

    # (OR,AND), pattern only, with kept bitmaps as benchmarked
    p = S.Product(Apat, Apat, "or_and_bool", B.make_options(bitmap_mib=28672))
    nnz_b = p.symbolic()
    C = p.numeric()
    assert p.stats()[0] == int(fl.sum())
    ptr_bool = C.ptr.cpu().numpy()
    got = _fetch(C, rows)
    _check_sorted_in_range(C, A.ncols)
    full_b = _check_every_row(C, Hpat, "or_and_bool", A.nrows)
    print(f"[fullsize] (OR,AND) every slice against the oracle's digests: {full_b}", flush=True)
    assert full_b, "the stored digests of the (OR,AND) square are missing"
    p.close()
    del C, p
    torch.cuda.empty_cache()
    assert_parity(Hpat, Hpat, "or_and_bool", got, select=rows,
                  want=oracle.spgemm(Hpat, Hpat, "or_and_bool", select=rows, nthreads=NTHREADS))

    # (min,+) int32 with the benchmarked kept-bitmap budget for its rank passes
    p = S.Product(dA, dA, "min_plus_i32", B.make_options(bitmap_mib=28672))
    nnz_m = p.symbolic()
    C = p.numeric()
    assert nnz_m == nnz_b
    assert np.array_equal(C.ptr.cpu().numpy(), ptr_bool), "the two semirings differ in pattern"
    # weights are in [1,255]: every 2-hop sum is in [2,510]
    for lo in range(0, nnz_m, 1 << 30):
        v = C.val[lo:lo + (1 << 30)]
        assert int(v.min()) >= 2 and int(v.max()) <= 510
    got = _fetch(C, rows)
    _check_sorted_in_range(C, A.ncols)
    full_m = _check_every_row(C, A, "min_plus_i32", A.nrows)
    print(f"[fullsize] (min,+) every slice against the oracle's digests: {full_m}", flush=True)
    assert full_m, "the stored digests of the (min,+) square are missing"
    p.close()
    del C, p
    torch.cuda.empty_cache()
    assert_parity(A, A, "min_plus_i32", got, select=rows,
                  want=oracle.spgemm(A, A, "min_plus_i32", select=rows, nthreads=NTHREADS))


# --------------------------------------------------------------------------
# MCL expansion n = 2^20, CSC float32, then prune
# --------------------------------------------------------------------------
def test_mcl_expansion_and_prune():
    import torch

    from paper_2106_14402_amd import spgemm as S
    A = spgen.config_mcl()
    fl = oracle.flops(A, A)
    cols = _sample(fl, np.random.default_rng(12), n_rand=96)
    print(f"[fullsize] MCL n=2^20 sample of {cols.size} columns", flush=True)
    dA = S.to_device(A)
    p = S.Product(dA, dA, "plus_times_f32")
    nnz = p.symbolic()
    C = p.numeric()
    assert int(C.idx.numel()) == nnz
    _check_sorted_in_range(C, A.nrows)
    # column sums of a product of column-stochastic matrices are 1
    cs = torch.cumsum(C.val.double(), 0)
    ends = cs[C.ptr[1:] - 1]
    starts = torch.cat([torch.zeros(1, dtype=torch.float64, device=cs.device), ends[:-1]])
    colsum = (ends - starts).cpu().numpy()
    del cs, ends, starts
    assert np.all(np.diff(C.ptr.cpu().numpy()) > 0)
    assert np.max(np.abs(colsum - 1.0)) < 1e-4
    got = _fetch(C, cols)
    # prune on the device: the kept count equals the count of values >= 1e-4
    P = S.prune_f32(C, 1e-4)
    keep = sum(int((C.val[lo:lo + (1 << 30)] >= 1e-4).sum()) for lo in range(0, nnz, 1 << 30))
    assert int(P.idx.numel()) == keep
    gotp = _fetch(P, cols)
    torch.cuda.synchronize()
    p.close()
    del C, P, p
    torch.cuda.empty_cache()

    want = oracle.spgemm(A, A, "plus_times_f32", select=cols, nthreads=NTHREADS)
    assert_parity(A, A, "plus_times_f32", got, select=cols, want=want)
    # pruned slices: exactly the GPU's own entries >= 1e-4 ...
    gp, gi, gv = got
    m = gv >= np.float32(1e-4)
    cm = np.concatenate([[0], np.cumsum(m, dtype=np.int64)])
    cnt = cm[gp[1:]] - cm[gp[:-1]]
    assert np.array_equal(np.diff(gotp[0]), cnt)
    assert np.array_equal(gotp[1], gi[m]) and np.array_equal(gotp[2], gv[m])
    # ... and against the float64 oracle only inside the tolerance band (all
    # values are nonnegative, so the (+,x) tolerance is 1e-5 of the value;
    # the float32 threshold differs from 1e-4 by less than 3e-12)
    _, oi, ov = want
    flip = m != (ov >= 1e-4)
    band = np.abs(ov - 1e-4) <= 1e-5 * ov + 3e-12
    assert not np.any(flip & ~band)


# --------------------------------------------------------------------------
# 512 uneven products, numeric phase replayed from the captured graph
# --------------------------------------------------------------------------
def test_batched_512_sampled():
    import torch

    from paper_2106_14402_amd import batch as BT
    from paper_2106_14402_amd import spgemm as S
    items = spgen.batch_mix()
    mats = [S.to_device(it.A) for it in items]
    srs = [it.semiring for it in items]
    bp = BT.BatchProduct(mats, mats, srs)
    bp.symbolic()
    bp.capture()
    bp.replay()
    bp.replay()
    torch.cuda.synchronize()
    rng = np.random.default_rng(13)
    prods = np.unique(np.concatenate([rng.choice(len(items), 24, replace=False),
                                      [0, len(items) - 1]]))
    print(f"[fullsize] batched: checking products {prods.tolist()}", flush=True)
    for b in prods:
        A, sr = items[b].A, srs[b]
        C = bp.result(int(b))
        fl = oracle.flops(A, A)
        rows = _sample(fl, np.random.default_rng(100 + int(b)), n_heavy=4, n_rand=32)
        got = _fetch(C, rows)
        assert_parity(A, A, sr, got, select=rows, want=oracle.spgemm(A, A, sr, select=rows, nthreads=NTHREADS))
    bp.close()


# --------------------------------------------------------------------------
# Served frontier expansion on the resident R-MAT scale 22 adjacency
# --------------------------------------------------------------------------
def test_served_s22_sampled():
    from paper_2106_14402_amd import serve as SV
    A = spgen.config_served_graph()
    g = SV.ResidentGraph(A)
    reqs = spgen.request_stream(A.nrows, 120, rate=4000.0, rng=spgen.rng_for(4, 3))
    res = SV.FrontierServer(g, workers=3).serve(reqs)
    assert all(r.status == SV.SPG_OK for r in res)
    assert any(r.batch_rows > q.k for q, r in zip(reqs, res))   # some requests shared a product
    rng = np.random.default_rng(14)
    for i in rng.choice(len(reqs), 12, replace=False):
        q, r = reqs[i], res[i]
        want = oracle.spgemm(q.Ft, A, "or_and_bool", nthreads=NTHREADS)
        assert np.array_equal(r.ptr, want[0]) and np.array_equal(r.idx, want[1])
        ap, ai = SV.expand_alone(g, q.Ft)
        assert np.array_equal(ap, r.ptr) and np.array_equal(ai, r.idx)
