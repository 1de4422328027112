"""Pins of the CPU oracle against facts fixed by mathematics (no GPU).

The paper prints no worked example and no per-matrix values that can be
reproduced here (its matrices are not available), so the oracle is pinned to:
dense brute force on tiny inputs (the definition of the product, Sec. 3.1),
exhaustive 3x3 boolean products, 2-hop reachability and 2-hop shortest walks
found by independent search, a library sparse product (scipy), the
column-stochastic invariant, the transposition identity (AB)^T = B^T A^T that
ties the column-wise (Sec. 4.1) and row-wise code paths together, semiring
identities, permutation equivariance and the exact flop count of the
Erdos-Renyi workload.
"""
import itertools
import math

import numpy as np
import pytest
import scipy.sparse as sp

import oracle
import spgen
from tests.semiring_ref import brute_force, to_dense_result

ALL = list(oracle.SEMIRINGS)
VALKIND = {"plus_times_f64": "f64", "plus_times_f32": "f32", "min_plus_i32": "i32",
           "min_plus_f32": "f32", "or_and_bool": "bool", "max_times_f64": "f64",
           "max_times_f32": "f32"}


def random_sparse(m, n, density, rng, kind, layout="csr", signed=False):
    nmajor, nminor = (m, n) if layout == "csr" else (n, m)
    degs = rng.binomial(nminor, density, size=nmajor)
    major, minor = spgen.distinct_minor(nmajor, nminor, degs, rng)
    val = spgen.draw_values(kind, major.size, rng)
    if val is not None and kind in ("f64", "f32"):
        if signed:
            val = (val - 0.5).astype(val.dtype)
        else:
            val = (val + 0.25).astype(val.dtype)
    if kind == "bool" and val is not None:
        val = rng.integers(0, 2, size=major.size).astype(np.uint8)  # explicit falses too
    if kind == "i32":
        val = rng.integers(-300, 300, size=major.size).astype(np.int32)
    return spgen.from_pairs(m, n, major, minor, val, layout, presorted=True)


def check_against_brute(A, B, sr, rtol=1e-13):
    ptr, idx, val = oracle.spgemm(A, B, sr)
    m, k = A.nrows, B.ncols
    nmajor, nminor = (m, k) if A.layout == "csr" else (k, m)
    pres, vals = to_dense_result(ptr, idx, val, nmajor, nminor, A.layout, val.dtype)
    bp, bv = brute_force(A, B, sr)
    assert np.array_equal(pres, bp), "pattern differs from the definition"
    if sr.startswith("plus_times"):
        Aa, Ba = A.with_values(np.abs(A.val)), B.with_values(np.abs(B.val))
        _, absv = brute_force(Aa, Ba, "plus_times_f64")
        assert np.all(np.abs(vals - bv) <= rtol * absv + 1e-300)
    else:
        assert np.array_equal(vals[bp].view(np.uint8), bv[bp].astype(vals.dtype).view(np.uint8)), \
            "values differ from the definition"


@pytest.mark.parametrize("sr", ALL)
@pytest.mark.parametrize("layout", ["csr", "csc"])
def test_dense_brute_force(sr, layout):
    rng = np.random.default_rng(7)
    for trial, (m, n, k, dens) in enumerate([(13, 17, 11, 0.3), (29, 23, 31, 0.15), (1, 40, 1, 0.5),
                                            (40, 1, 40, 0.5), (20, 20, 20, 0.9)]):
        A = random_sparse(m, n, dens, rng, VALKIND[sr], layout, signed=True)
        B = random_sparse(n, k, dens, rng, VALKIND[sr], layout, signed=True)
        check_against_brute(A, B, sr)


def test_pattern_only_bool_equals_all_true():
    rng = np.random.default_rng(8)
    A = random_sparse(30, 25, 0.2, rng, None)
    B = random_sparse(25, 35, 0.2, rng, None)
    check_against_brute(A, B, "or_and_bool")
    p1, i1, v1 = oracle.spgemm(A, B, "or_and_bool")
    p2, i2, v2 = oracle.spgemm(A.with_values(np.ones(A.nnz, np.uint8)),
                               B.with_values(np.ones(B.nnz, np.uint8)), "or_and_bool")
    assert np.array_equal(p1, p2) and np.array_equal(i1, i2) and np.array_equal(v1, v2)
    assert np.all(v1 == 1)


def _mat3(bits):
    rows, cols = [], []
    for r in range(3):
        for c in range(3):
            if bits >> (3 * r + c) & 1:
                rows.append(r)
                cols.append(c)
    return rows, cols


def test_exhaustive_3x3_boolean():
    """All 512 x 512 pairs of 3x3 boolean patterns (pattern and values).

    512 block-diagonal products cover every pair: call r multiplies
    diag(A_0..A_511) by diag(B_{(t+r) mod 512})."""
    dense = np.zeros((512, 3, 3), bool)
    for t in range(512):
        r, c = _mat3(t)
        dense[t, r, c] = True
    expect = (dense[:, None, :, :, None] & dense[None, :, None, :, :]).any(axis=3)  # (a, b, 3, 3)
    rows_a, cols_a = [], []
    for t in range(512):
        r, c = _mat3(t)
        rows_a += [3 * t + x for x in r]
        cols_a += [3 * t + x for x in c]
    N = 1536
    A = spgen.from_pairs(N, N, np.array(rows_a), np.array(cols_a), None)
    L = oracle.lib()
    for shift in range(512):
        rows_b, cols_b = [], []
        for t in range(512):
            r, c = _mat3((t + shift) % 512)
            rows_b += [3 * t + x for x in r]
            cols_b += [3 * t + x for x in c]
        B = spgen.from_pairs(N, N, np.array(rows_b), np.array(cols_b), None)
        ptr, idx, val = oracle.spgemm(A, B, "or_and_bool", nthreads=1, _lib=L)
        assert np.all(val == 1)
        got = np.zeros((N, 3), bool)
        row_of = np.repeat(np.arange(N), np.diff(ptr))
        assert np.all(idx // 3 == row_of // 3), "product leaked across blocks"
        got[row_of, idx % 3] = True
        got = got.reshape(512, 3, 3)
        want = expect[np.arange(512), (np.arange(512) + shift) % 512]
        assert np.array_equal(got, want), f"shift {shift}"


def test_boolean_square_is_two_hop_walks():
    rng = np.random.default_rng(11)
    n = 300
    A = spgen.rmat_graph(0, 4, rng, symmetric=False, n=n)
    adj = [set(A.idx[A.ptr[i]:A.ptr[i + 1]].tolist()) for i in range(n)]
    ptr, idx, _ = oracle.spgemm(A, A, "or_and_bool")
    for i in range(n):
        walk2 = set()
        for k in adj[i]:                       # breadth-first, exactly two levels
            walk2 |= adj[k]
        assert set(idx[ptr[i]:ptr[i + 1]].tolist()) == walk2


def test_min_plus_square_is_two_hop_shortest_walk():
    rng = np.random.default_rng(12)
    n = 80
    A = spgen.rmat_graph(0, 6, rng, symmetric=True, weights="i32", n=n)
    w = {}
    for i in range(n):
        for p in range(A.ptr[i], A.ptr[i + 1]):
            w[(i, int(A.idx[p]))] = int(A.val[p])
    ptr, idx, val = oracle.spgemm(A, A, "min_plus_i32")
    got = {(i, int(idx[p])): int(val[p]) for i in range(n) for p in range(ptr[i], ptr[i + 1])}
    want = {}
    for i in range(n):                          # exhaustive over every intermediate vertex
        for j in range(n):
            best = None
            for k in range(n):
                if (i, k) in w and (k, j) in w:
                    d = w[(i, k)] + w[(k, j)]
                    best = d if best is None else min(best, d)
            if best is not None:
                want[(i, j)] = best
    assert got == want
    # symmetric weights: the square is symmetric too
    assert all(got[(j, i)] == v for (i, j), v in got.items())


def test_plus_times_matches_scipy():
    A = spgen.config_er()
    ptr, idx, val = oracle.spgemm(A, A, "plus_times_f64")
    S = sp.csr_matrix((A.val, A.idx, A.ptr), shape=(A.nrows, A.ncols))
    C = (S @ S).tocsr()
    C.sort_indices()
    assert np.array_equal(C.indptr, ptr)
    assert np.array_equal(C.indices, idx)
    assert np.allclose(C.data, val, rtol=1e-13, atol=0)


def test_er_flop_count_and_expected_output_size():
    A = spgen.config_er()
    f = oracle.flops(A, A)
    assert int(f.sum()) == 4096 * 8 * 8          # every row: 8 rows of B with 8 entries each
    assert np.all(f == 64)
    ptr, _, _ = oracle.spgemm(A, A, "plus_times_f64")
    n, d = 4096, 8
    # A column is missed by one B row (d of n without replacement) with
    # probability 1 - d/n, and by all d rows independently.
    expect = n * n * (1 - (1 - d / n) ** d)
    assert abs(ptr[-1] - expect) / expect < 0.01


def test_column_stochastic_invariant():
    rng = np.random.default_rng(13)
    A = spgen.mcl_matrix(3000, 12.0, 1.0, rng)
    ptr, idx, val = oracle.spgemm(A, A, "plus_times_f32")
    n = A.ncols
    colA = np.bincount(np.repeat(np.arange(n), np.diff(A.ptr)), weights=A.val.astype(np.float64),
                       minlength=n)
    # colsum(C)_j = sum_k colsum(A)_k A(k,j)
    col_of = np.repeat(np.arange(n), np.diff(A.ptr))
    want = np.bincount(col_of, weights=colA[A.idx] * A.val.astype(np.float64), minlength=n)
    got = np.add.reduceat(val, ptr[:-1]) if val.size else np.zeros(n)
    got = np.where(np.diff(ptr) > 0, got, 0.0)
    assert np.allclose(got, want, rtol=1e-12, atol=0)
    assert np.allclose(got, 1.0, atol=1e-5)


def _to_layout(M, layout):
    """Same matrix in the other storage layout (explicit re-packing)."""
    if M.layout == layout:
        return M
    major = np.repeat(np.arange(M.nmajor), np.diff(M.ptr))
    minor = M.idx.astype(np.int64)
    # old (major, minor) -> new: roles swap
    return spgen.from_pairs(M.nrows, M.ncols, minor, major, M.val, layout)


def _transpose(M):
    """Explicit transpose, same layout."""
    T = M.transpose_view()
    return _to_layout(T, M.layout)


@pytest.mark.parametrize("sr", ALL)
def test_csc_path_equals_csr_path_and_transpose_identity(sr):
    rng = np.random.default_rng(14)
    A = random_sparse(60, 45, 0.1, rng, VALKIND[sr], signed=True)
    B = random_sparse(45, 70, 0.1, rng, VALKIND[sr], signed=True)
    p, i, v = oracle.spgemm(A, B, sr)
    # column-wise Gustavson on the CSC copies
    pc, ic, vc = oracle.spgemm(_to_layout(A, "csc"), _to_layout(B, "csc"), sr)
    C = spgen.from_pairs(60, 70, np.repeat(np.arange(60), np.diff(p)), i, v)
    Cc = _to_layout(spgen.SparseMatrix(60, 70, "csc", pc, ic, vc), "csr")
    assert np.array_equal(C.ptr, Cc.ptr) and np.array_equal(C.idx, Cc.idx)
    assert np.array_equal(C.val, Cc.val)
    # (AB)^T = B^T A^T  (all listed multiplications are commutative)
    pt, it, vt = oracle.spgemm(_transpose(B), _transpose(A), sr)
    Ct = _transpose(C)
    assert np.array_equal(Ct.ptr, pt) and np.array_equal(Ct.idx, it)
    if sr.startswith("plus_times"):
        assert np.allclose(Ct.val, vt, rtol=1e-12, atol=1e-14)
    else:
        assert np.array_equal(Ct.val, vt)


MUL_IDENTITY = {"plus_times_f64": 1.0, "plus_times_f32": 1.0, "min_plus_i32": 0, "min_plus_f32": 0.0,
                "or_and_bool": 1, "max_times_f64": 1.0, "max_times_f32": 1.0}


@pytest.mark.parametrize("sr", ALL)
def test_identity_matrix(sr):
    rng = np.random.default_rng(15)
    A = random_sparse(50, 50, 0.08, rng, VALKIND[sr], signed=True)
    ident = spgen.from_pairs(50, 50, np.arange(50), np.arange(50),
                             np.full(50, MUL_IDENTITY[sr], dtype=A.val.dtype))
    for X, Y in ((A, ident), (ident, A)):
        p, i, v = oracle.spgemm(X, Y, sr)
        assert np.array_equal(p, A.ptr) and np.array_equal(i, A.idx)
        assert np.array_equal(v, A.val.astype(v.dtype))


@pytest.mark.parametrize("sr", ["min_plus_i32", "or_and_bool", "plus_times_f64"])
def test_permutation_equivariance(sr):
    rng = np.random.default_rng(16)
    n = 120
    A = spgen.rmat_graph(0, 5, rng, symmetric=False, n=n,
                         weights={"min_plus_i32": "i32", "or_and_bool": None, "plus_times_f64": "f64"}[sr])
    perm = rng.permutation(n)
    rows = np.repeat(np.arange(n), np.diff(A.ptr))
    PA = spgen.from_pairs(n, n, perm[rows], perm[A.idx], A.val)
    p, i, v = oracle.spgemm(A, A, sr)
    pp, ip, vp = oracle.spgemm(PA, PA, sr)
    rowsC = np.repeat(np.arange(n), np.diff(p))
    PC = spgen.from_pairs(n, n, perm[rowsC], perm[i], v)
    assert np.array_equal(PC.ptr, pp) and np.array_equal(PC.idx, ip)
    if sr == "plus_times_f64":
        assert np.allclose(PC.val, vp, rtol=1e-12)
    else:
        assert np.array_equal(PC.val, vp)


def test_min_plus_i32_saturates():
    big = np.iinfo(np.int32).max
    A = spgen.from_pairs(1, 2, np.array([0, 0]), np.array([0, 1]), np.array([big - 5, -big], np.int32))
    B = spgen.from_pairs(2, 2, np.array([0, 1]), np.array([0, 1]), np.array([100, -100], np.int32))
    p, i, v = oracle.spgemm(A, B, "min_plus_i32")
    # (big-5)+100 clamps to INT32_MAX; -big + -100 clamps to INT32_MIN
    assert list(i) == [0, 1] and list(v) == [big, np.iinfo(np.int32).min]


def test_signed_zero_total_order():
    # (min,+): -0 + -0 = -0 and +0 + +0 = +0 meet in one entry; min is -0.
    A = spgen.from_pairs(1, 2, np.array([0, 0]), np.array([0, 1]), np.array([0.0, -0.0], np.float32))
    B = spgen.from_pairs(2, 1, np.array([0, 1]), np.array([0, 0]), np.array([0.0, -0.0], np.float32))
    _, _, v = oracle.spgemm(A, B, "min_plus_f32")
    assert v[0] == 0 and np.signbit(v[0])
    for sr, dt in (("max_times_f32", np.float32), ("max_times_f64", np.float64)):
        # (max,x): 1 * -0 = -0 and 1 * +0 = +0; max is +0 whichever comes first.
        for order in ([-0.0, 0.0], [0.0, -0.0]):
            A = spgen.from_pairs(1, 2, np.array([0, 0]), np.array([0, 1]), np.array([1.0, 1.0], dt))
            B = spgen.from_pairs(2, 1, np.array([0, 1]), np.array([0, 0]), np.array(order, dt))
            _, _, v = oracle.spgemm(A, B, sr)
            assert v[0] == 0 and not np.signbit(v[0])


def test_structural_identity_results_are_kept():
    # (+,x): 1*0.5 + (-1)*0.5 = 0 is still stored (structural pattern).
    A = spgen.from_pairs(1, 2, np.array([0, 0]), np.array([0, 1]), np.array([1.0, -1.0]))
    B = spgen.from_pairs(2, 1, np.array([0, 1]), np.array([0, 0]), np.array([0.5, 0.5]))
    p, i, v = oracle.spgemm(A, B, "plus_times_f64")
    assert list(p) == [0, 1] and v[0] == 0.0
    # (OR,AND): explicit false operands still produce a stored (false) entry.
    A = spgen.from_pairs(1, 1, np.array([0]), np.array([0]), np.array([0], np.uint8))
    B = spgen.from_pairs(1, 1, np.array([0]), np.array([0]), np.array([1], np.uint8))
    p, i, v = oracle.spgemm(A, B, "or_and_bool")
    assert list(p) == [0, 1] and v[0] == 0


def test_empty_operands():
    E = spgen.from_pairs(5, 7, np.array([], np.int64), np.array([], np.int64), np.array([], np.float64))
    F = random_sparse(7, 3, 0.5, np.random.default_rng(1), "f64")
    p, i, v = oracle.spgemm(E, F, "plus_times_f64")
    assert list(p) == [0] * 6 and i.size == 0
    Z = spgen.from_pairs(0, 7, np.array([], np.int64), np.array([], np.int64), np.array([], np.float64))
    p, i, v = oracle.spgemm(Z, F, "plus_times_f64")
    assert list(p) == [0] and i.size == 0


def test_prune_by_brute_force():
    rng = np.random.default_rng(17)
    A = random_sparse(40, 30, 0.3, rng, "f32")
    vals = (rng.random(A.nnz) * 2e-4).astype(np.float32)
    vals[::7] = np.float32(1e-4)                  # the boundary is kept (>=)
    p, i, v = oracle.prune_f32(A.ptr, A.idx, vals, 1e-4)
    thr = np.float32(1e-4)
    for r in range(A.nrows):
        lo, hi = A.ptr[r], A.ptr[r + 1]
        keep = [(int(c), x) for c, x in zip(A.idx[lo:hi], vals[lo:hi]) if x >= thr]
        assert [c for c, _ in keep] == i[p[r]:p[r + 1]].tolist()
        assert [x for _, x in keep] == v[p[r]:p[r + 1]].tolist()
