"""Pins of the oracle's slice digests, its CSC flop count and its selection.

The digests let the whole output of a product too large to hold be compared
slice by slice with the definition C = AB (paper Sec. 3.1).  They are pinned
here against SplitMix64's published outputs, against a hand-derived product,
and against the oracle's own product (pinned elsewhere) hashed independently
in Python.
"""
import numpy as np
import pytest

import oracle
import spgen

M64 = (1 << 64) - 1


def mix64_py(z: int) -> int:
    z &= M64
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & M64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & M64
    return z ^ (z >> 31)


def slice_digest_py(ids, vbits) -> int:
    h = 0
    for t, (j, v) in enumerate(zip(ids, vbits)):
        h = (h + mix64_py(mix64_py((t << 32) | int(j)) ^ int(v))) & M64
    return h


def vbits_of(vals) -> list:
    a = np.ascontiguousarray(vals)
    if a.dtype.itemsize == 8:
        return [int(x) for x in a.view(np.uint64)]
    if a.dtype.itemsize == 4:
        return [int(x) for x in a.view(np.uint32)]
    return [int(x) for x in a.view(np.uint8)]


def test_mix64_matches_splitmix64_published_outputs():
    # SplitMix64 seeded with 0 returns mix64(k * 0x9E3779B97F4A7C15) as its
    # k-th output; its first two are 0xE220A8397B1DCDAF and 0x6E789E6AA1B965F4.
    g = 0x9E3779B97F4A7C15
    got = oracle.mix64(np.array([g, (2 * g) & M64], np.uint64))
    assert [int(x) for x in got] == [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4]
    xs = np.random.default_rng(0).integers(0, 2**63, size=50, dtype=np.int64).astype(np.uint64)
    assert [int(x) for x in oracle.mix64(xs)] == [mix64_py(int(x)) for x in xs]


def test_digest_hand_computed_min_plus():
    # A = [1 2] (1 x 2), B = [[., 3], [4, .]] over (min,+):
    # C(0,0) = 2 + 4 = 6 (only k = 1), C(0,1) = 1 + 3 = 4 (only k = 0).
    A = spgen.SparseMatrix(1, 2, "csr", np.array([0, 2], np.int64), np.array([0, 1], np.int32),
                           np.array([1, 2], np.int32))
    B = spgen.SparseMatrix(2, 2, "csr", np.array([0, 1, 2], np.int64), np.array([1, 0], np.int32),
                           np.array([3, 4], np.int32))
    nnz, h = oracle.digest(A, B, "min_plus_i32")
    want = (mix64_py(mix64_py(0) ^ 6) + mix64_py(mix64_py((1 << 32) | 1) ^ 4)) & M64
    assert nnz.tolist() == [2] and int(h[0]) == want
    # the same two entries in the other order (a wrong sort) would not match
    swapped = (mix64_py(mix64_py(1) ^ 4) + mix64_py(mix64_py((1 << 32) | 0) ^ 6)) & M64
    assert swapped != want


@pytest.mark.parametrize("sr", ["min_plus_i32", "min_plus_f32", "or_and_bool", "max_times_f64",
                                "max_times_f32"])
@pytest.mark.parametrize("layout", ["csr", "csc"])
def test_digest_equals_hash_of_oracle_product(sr, layout):
    rng = np.random.default_rng(11)
    kinds = {"min_plus_i32": "i32", "min_plus_f32": "f32", "or_and_bool": "bool",
             "max_times_f64": "f64", "max_times_f32": "f32"}
    A = spgen.rmat_graph(0, 6, rng, symmetric=False, weights=kinds[sr], n=300)
    B = spgen.rmat_graph(0, 6, rng, symmetric=False, weights=kinds[sr], n=300)
    if layout == "csc":
        A, B = A.transpose_view(), B.transpose_view()
    ptr, idx, val = oracle.spgemm(A, B, sr)
    nnz, h = oracle.digest(A, B, sr)
    assert np.array_equal(nnz, np.diff(ptr))
    for s in range(0, nnz.size, 7):
        lo, hi = int(ptr[s]), int(ptr[s + 1])
        assert int(h[s]) == slice_digest_py(idx[lo:hi], vbits_of(val[lo:hi]))
    sel = np.array([5, 3, 250], np.int64)
    n2, h2 = oracle.digest(A, B, sr, select=sel)
    assert np.array_equal(n2, nnz[sel]) and np.array_equal(h2, h[sel])


def test_digest_rejects_plus_times():
    A = spgen.config_er(n=64, d=4)
    with pytest.raises(ValueError):
        oracle.digest(A, A, "plus_times_f64")


def test_block_digests_definition():
    rng = np.random.default_rng(3)
    nnz = rng.integers(0, 50, size=2500).astype(np.int64)
    h = rng.integers(0, 2**63, size=2500, dtype=np.int64).astype(np.uint64)
    bn, bh = oracle.block_digests(nnz, h, first_slice=1024, block=1000)
    assert bn.size == 3 and bh.size == 3
    for b in range(3):
        want_h, want_n = 0, 0
        for t in range(b * 1000, min(2500, (b + 1) * 1000)):
            i = 1024 + t
            want_h = (want_h + mix64_py(int(h[t]) ^ mix64_py((i << 32) | int(nnz[t])))) & M64
            want_n += int(nnz[t])
        assert int(bh[b]) == want_h and int(bn[b]) == want_n


def brute_flops_rows(A, B):
    """Products per row of A*B (CSR), counted by walking dense copies."""
    Ad = np.zeros((A.nrows, A.ncols), bool)
    Bd = np.zeros((B.nrows, B.ncols), bool)
    for i in range(A.nrows):
        Ad[i, A.idx[A.ptr[i]:A.ptr[i + 1]]] = True
    for k in range(B.nrows):
        Bd[k, B.idx[B.ptr[k]:B.ptr[k + 1]]] = True
    return np.array([sum(int(Bd[k].sum()) for k in np.nonzero(Ad[i])[0]) for i in range(A.nrows)])


def test_csc_flops_pinned():
    rng = np.random.default_rng(21)
    for _ in range(3):
        A = spgen.erdos_renyi(40, 5, rng, values="f64", ncols=30)
        B = spgen.erdos_renyi(30, 7, rng, values="f64", ncols=50)
        # CSR: brute force per row of C
        assert np.array_equal(oracle.flops(A, B), brute_flops_rows(A, B))
        # CSC view of the transposes: C^T = B^T A^T column by column has the
        # same products per slice as the CSR rows of C = A B
        At, Bt = A.transpose_view(), B.transpose_view()   # CSC arrays of A^T, B^T
        assert np.array_equal(oracle.flops(Bt, At), brute_flops_rows(A, B))
        # a CSC product counted directly: slice j of X Y (X m x n, Y n x k,
        # both CSC) takes nnz(X(:,l)) products per stored Y(l,j)
        X, Y = B.transpose_view(), A.transpose_view()
        want = np.array([sum(int(X.ptr[l + 1] - X.ptr[l]) for l in Y.idx[Y.ptr[j]:Y.ptr[j + 1]])
                         for j in range(Y.ncols)])
        assert np.array_equal(oracle.flops(X, Y), want)


def test_select_hand_computed_column():
    # one column: ids 1 3 4 7 9, values .1 .5 .2 .5 .4; S = 3 keeps .5 (3), .5 (7), .4 (9)
    ptr = np.array([0, 5], np.int64)
    idx = np.array([1, 3, 4, 7, 9], np.int32)
    val = np.array([0.1, 0.5, 0.2, 0.5, 0.4], np.float32)
    p, i, v = oracle.select_f32(ptr, idx, val, 3)
    assert p.tolist() == [0, 3] and i.tolist() == [3, 7, 9]
    assert v.tolist() == pytest.approx([0.5, 0.5, 0.4])
    # a tie at the cut goes to the smaller id: S = 1 keeps id 3, not 7
    p, i, v = oracle.select_f32(ptr, idx, val, 1)
    assert i.tolist() == [3]
    # -0 < +0: S = 1 of (+0 at id 2, -0 at id 0) keeps id 2
    p, i, v = oracle.select_f32(np.array([0, 2], np.int64), np.array([0, 2], np.int32),
                                np.array([-0.0, 0.0], np.float32), 1)
    assert i.tolist() == [2] and not np.signbit(v[0])


def test_select_identity_and_bounds():
    A = spgen.config_mcl(n=2000, mean_deg=20.0)
    longest = int(np.diff(A.ptr).max())
    p, i, v = oracle.select_f32(A.ptr, A.idx, A.val, longest)
    assert np.array_equal(p, A.ptr) and np.array_equal(i, A.idx) and np.array_equal(v, A.val)
    S = 7
    p, i, v = oracle.select_f32(A.ptr, A.idx, A.val, S)
    assert np.array_equal(np.diff(p), np.minimum(np.diff(A.ptr), S))
    for s in range(0, A.ncols, 37):
        lo, hi = int(A.ptr[s]), int(A.ptr[s + 1])
        kept = i[p[s]:p[s + 1]]
        assert np.all(np.diff(kept) > 0)
        if hi - lo > S:
            # every dropped value is <= every kept value
            dropped = np.setdiff1d(A.idx[lo:hi], kept)
            vmap = dict(zip(A.idx[lo:hi].tolist(), A.val[lo:hi].tolist()))
            assert max(vmap[d] for d in dropped) <= min(vmap[k] for k in kept.tolist())
