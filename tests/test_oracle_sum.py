"""Pins of the oracle's semiring sum (the merge of partial products), CPU only.

* the definition written out densely: every entry of the result is the (+)
  of the parts that hold it, absent where no part holds it;
* Sparse SUMMA's identity: splitting the inner dimension of A B into k
  blocks, the sum of the k partial products A(:,K_t) B(K_t,:) is A B (this
  ties the sum to the oracle's product, an independent code path);
* one part is returned unchanged;
* planted mistakes in the sum's source fail these pins.
"""
import os
import subprocess

import numpy as np
import pytest

import oracle
import spgen
from tests.test_oracle_pins import ALL, VALKIND, random_sparse
from tests.semiring_ref import to_dense_result

EXACT = [s for s in ALL if not s.startswith("plus_times")]


def _dense_parts(parts):
    """(presence[k, m, n], values[k, m, n]) in row/column orientation."""
    k = len(parts)
    m, n = parts[0].nrows, parts[0].ncols
    pres = np.zeros((k, m, n), bool)
    vals = np.zeros((k, m, n), object)
    for t, P in enumerate(parts):
        for s in range(P.ptr.size - 1):
            for q in range(P.ptr[s], P.ptr[s + 1]):
                i, j = (s, P.idx[q]) if P.layout == "csr" else (P.idx[q], s)
                pres[t, i, j] = True
                vals[t, i, j] = 1 if P.val is None else P.val[q]
    return pres, vals


def _fold(sr, xs):
    """(+) of a list of values, written from the semiring's definition."""
    if sr.startswith("plus_times"):
        return float(sum(float(x) for x in xs))
    if sr == "or_and_bool":
        return int(any(int(x) != 0 for x in xs))
    if sr.startswith("min_plus"):
        return min(xs)
    return max(xs)


def _check_sum(parts, sr):
    ptr, idx, val = oracle.sum_parts(parts, sr)
    m, n = parts[0].nrows, parts[0].ncols
    nmaj, nmin = (m, n) if parts[0].layout == "csr" else (n, m)
    pres, vals = to_dense_result(ptr, idx, val, nmaj, nmin, parts[0].layout, val.dtype)
    pp, pv = _dense_parts(parts)
    want_pres = pp.any(axis=0)
    assert np.array_equal(pres, want_pres), "pattern is not the union of the parts"
    for i, j in zip(*np.nonzero(want_pres)):
        xs = [pv[t, i, j] for t in range(len(parts)) if pp[t, i, j]]
        w = _fold(sr, xs)
        if sr.startswith("plus_times"):
            assert abs(float(vals[i, j]) - w) <= 1e-12 * sum(abs(float(x)) for x in xs)
        else:
            assert vals[i, j] == w


@pytest.mark.parametrize("sr", ALL)
@pytest.mark.parametrize("layout", ["csr", "csc"])
@pytest.mark.parametrize("k", [1, 2, 4])
def test_sum_equals_definition(sr, layout, k):
    rng = np.random.default_rng(31 + k)
    parts = [random_sparse(9, 11, 0.3, rng, VALKIND[sr], layout) for _ in range(k)]
    _check_sum(parts, sr)


def test_sum_of_one_part_is_the_part():
    rng = np.random.default_rng(5)
    P = random_sparse(20, 17, 0.2, rng, "i32")
    ptr, idx, val = oracle.sum_parts([P], "min_plus_i32")
    assert np.array_equal(ptr, P.ptr) and np.array_equal(idx, P.idx) and np.array_equal(val, P.val)


def _col_block(M, lo, hi):
    """Columns [lo, hi) of a CSR matrix, column ids kept (same shape)."""
    keep = (M.idx >= lo) & (M.idx < hi)
    rows = np.repeat(np.arange(M.nrows), np.diff(M.ptr))[keep]
    return spgen.from_pairs(M.nrows, M.ncols, rows, M.idx[keep], None if M.val is None else M.val[keep])


def _row_block(M, lo, hi):
    """Rows [lo, hi) of a CSR matrix (same shape, other rows empty)."""
    rows = np.repeat(np.arange(M.nrows), np.diff(M.ptr))
    keep = (rows >= lo) & (rows < hi)
    return spgen.from_pairs(M.nrows, M.ncols, rows[keep], M.idx[keep], None if M.val is None else M.val[keep])


@pytest.mark.parametrize("sr", ALL)
def test_summa_identity(sr):
    """A B = (+)_t A(:,K_t) B(K_t,:) for a split of the inner dimension."""
    rng = np.random.default_rng(41)
    A = random_sparse(30, 40, 0.15, rng, VALKIND[sr])
    B = random_sparse(40, 25, 0.15, rng, VALKIND[sr])
    cuts = [0, 7, 19, 33, 40]
    parts = []
    for lo, hi in zip(cuts[:-1], cuts[1:]):
        pp, pi, pv = oracle.spgemm(_col_block(A, lo, hi), _row_block(B, lo, hi), sr)
        val = None if sr == "or_and_bool" and A.val is None else pv
        if sr == "plus_times_f32":
            val = pv.astype(np.float32)  # the parts a float32 product would hold
        parts.append(spgen.SparseMatrix(30, 25, "csr", pp, pi, val))
    sp, si, sv = oracle.sum_parts(parts, sr)
    fp, fi, fv = oracle.spgemm(A, B, sr)
    assert np.array_equal(sp, fp) and np.array_equal(si, fi)
    if sr == "plus_times_f64":
        np.testing.assert_allclose(sv, fv, rtol=1e-12, atol=1e-12)
    elif sr == "plus_times_f32":
        np.testing.assert_allclose(sv, fv, rtol=1e-6, atol=1e-6)
    else:
        assert np.array_equal(sv.view(np.uint8), fv.view(np.uint8))


SUM_MUTANTS = {
    "sum_last_part_dropped": ("for (int t = 0; t < k; ++t) {", "for (int t = 0; t + 1 < k; ++t) {"),
    "sum_overwrites": ("        it->second = S::add(it->second, v);\n    }\n  }\n  keys.clear();",
                       "        it->second = v;\n    }\n  }\n  keys.clear();"),
    "sum_wrong_stride": ("const int64_t r = t * m + s;", "const int64_t r = t + s;"),
}


def _sum_pins_pass(L) -> bool:
    rng = np.random.default_rng(9)
    try:
        for sr in ("plus_times_f64", "min_plus_i32", "or_and_bool"):
            parts = [random_sparse(8, 9, 0.4, rng, VALKIND[sr]) for _ in range(3)]
            ptr, idx, val = oracle.sum_parts(parts, sr, _lib=L)
            pres, vals = to_dense_result(ptr, idx, val, 8, 9, "csr", val.dtype)
            pp, pv = _dense_parts(parts)
            if not np.array_equal(pres, pp.any(axis=0)):
                return False
            for i, j in zip(*np.nonzero(pres)):
                xs = [pv[t, i, j] for t in range(3) if pp[t, i, j]]
                w = _fold(sr, xs)
                if sr.startswith("plus_times"):
                    if abs(float(vals[i, j]) - w) > 1e-12 * sum(abs(float(x)) for x in xs):
                        return False
                elif vals[i, j] != w:
                    return False
    except (AssertionError, ValueError, IndexError):
        return False
    return True


@pytest.mark.parametrize("name", sorted(SUM_MUTANTS))
def test_sum_mutant_is_caught(name, tmp_path):
    assert _sum_pins_pass(oracle.lib())
    src = open(oracle.SRC).read()
    old, new = SUM_MUTANTS[name]
    assert src.count(old) == 1, f"mutation site for {name} not found"
    cpp = os.path.join(tmp_path, "mutant.cpp")
    so = os.path.join(tmp_path, f"libmutant_{name}.so")
    with open(cpp, "w") as f:
        f.write(src.replace(old, new))
    subprocess.check_call(["g++", "-O1", "-std=c++17", "-fopenmp", "-ffp-contract=off", "-fPIC",
                           "-shared", cpp, "-o", so])
    assert not _sum_pins_pass(oracle.load(so)), f"pins did not catch mutant {name}"
