"""Operands whose slices are not sorted (the paper's local matrices promise
no order, Sec. 2.1): the symbolic phase finds them with its operand check and
sorts them into the workspace, so every accumulator path (hash tables,
bitmaps, panel and chunk indexes, rank passes, kept bitmaps) sees sorted
slices.  Each product is compared with the oracle on the same entries (the
definition of C does not depend on the order of the entries)."""
import numpy as np
import pytest

import oracle
import spgen
from tests.gpu_util import assert_parity, run_gpu, with_semiring_values

pytestmark = pytest.mark.gpu


def opts(**kw):
    from paper_2106_14402_amd import binding
    return binding.make_options(**kw)


def shuffled(M, rng):
    """The same entries with every slice in a random order."""
    idx = M.idx.copy()
    val = None if M.val is None else M.val.copy()
    for s in range(M.ptr.size - 1):
        lo, hi = int(M.ptr[s]), int(M.ptr[s + 1])
        if hi - lo > 1:
            perm = lo + rng.permutation(hi - lo)
            idx[lo:hi] = M.idx[perm]
            if val is not None:
                val[lo:hi] = M.val[perm]
    return spgen.SparseMatrix(M.nrows, M.ncols, M.layout, M.ptr, idx, val)


def _skewed(n, ef, seed, symmetric=False):
    return spgen.rmat_graph(0, ef, np.random.default_rng(seed), symmetric=symmetric, n=n)


@pytest.mark.parametrize("which", ["both", "a", "b"])
def test_er_plus_times_f64(which):
    rng = np.random.default_rng(1)
    A = spgen.config_er()
    Au = shuffled(A, rng) if which in ("both", "a") else A
    Bu = shuffled(A, rng) if which in ("both", "b") else A
    got = run_gpu(Au, Bu, "plus_times_f64")
    assert_parity(A, A, "plus_times_f64", got)


@pytest.mark.parametrize("mode", ["default", "all_dense", "rank_kept", "many_panels", "fixed_chunks"])
def test_rmat_min_plus_paths(mode):
    rng = np.random.default_rng(2)
    A = with_semiring_values(_skewed(5000, 10, 4), "min_plus_i32", np.random.default_rng(5))
    o = {"default": None,
         "all_dense": opts(hash_max_flops=32, hash_max_nnz=32),
         "rank_kept": opts(hash_max_flops=32, hash_max_nnz=32, lds_budget=1024, dense_threads=256, bitmap_mib=1),
         "many_panels": opts(hash_max_flops=32, hash_max_nnz=32, sym_panel_log2=8, lds_budget=1024,
                             dense_threads=256, split_panels=1),
         "fixed_chunks": opts(hash_max_flops=32, hash_max_nnz=32, sym_panel_log2=8, lds_budget=1024,
                              rank_dense_div=100000)}[mode]
    got = run_gpu(shuffled(A, rng), shuffled(A, rng), "min_plus_i32", o)
    assert_parity(A, A, "min_plus_i32", got)


@pytest.mark.parametrize("sr", ["min_plus_i32", "plus_times_f64", "or_and_bool"])
def test_rank_passes_default_widths(sr):
    """70,000 columns: heavy rows take rank passes over the chunk index of the
    sorted copy of B (and kept bitmaps)."""
    rng = np.random.default_rng(3)
    A = with_semiring_values(_skewed(70000, 2, 21, symmetric=True), sr, np.random.default_rng(22))
    got = run_gpu(shuffled(A, rng), shuffled(A, rng), sr, opts(bitmap_mib=64))
    assert_parity(A, A, sr, got)


def test_pattern_only_kept_bitmaps():
    rng = np.random.default_rng(4)
    A = _skewed(7000, 14, 6)
    got = run_gpu(shuffled(A, rng), shuffled(A, rng), "or_and_bool", opts(bitmap_mib=1, hash_max_flops=64))
    assert_parity(A, A, "or_and_bool", got)


def test_mcl_csc_plus_times_f32():
    rng = np.random.default_rng(5)
    A = spgen.config_mcl(n=20000, mean_deg=24.0)
    got = run_gpu(shuffled(A, rng), shuffled(A, rng), "plus_times_f32")
    assert_parity(A, A, "plus_times_f32", got)


def test_long_slices_global_sort():
    """Slices longer than the LDS sort (2,048 ids) take the global-memory
    network: a few rows of 3,000-20,000 entries."""
    rng = np.random.default_rng(6)
    n = 30000
    degs = np.full(n, 3)
    degs[[5, 77, 1234]] = [3000, 9000, 20000]
    rows, cols = spgen.distinct_minor(n, n, degs, rng)
    A = spgen.from_pairs(n, n, rows, cols, rng.integers(1, 256, size=rows.size).astype(np.int32))
    got = run_gpu(shuffled(A, rng), shuffled(A, rng), "min_plus_i32")
    assert_parity(A, A, "min_plus_i32", got)


def test_sum_of_shuffled_parts():
    import torch
    from paper_2106_14402_amd import spgemm as S
    rng = np.random.default_rng(7)
    parts = [with_semiring_values(_skewed(3000, 6, 30 + t), "min_plus_i32", rng) for t in range(3)]
    want = oracle.sum_parts(parts, "min_plus_i32")
    C = S.spg_sum([S.to_device(shuffled(x, rng)) for x in parts], "min_plus_i32")
    torch.cuda.synchronize()
    got = (C.ptr.cpu().numpy(), C.idx.cpu().numpy(), C.val.cpu().numpy())
    assert_parity(None, None, "min_plus_i32", got, want=want)


def test_sort_rejected_without_room_and_duplicates():
    import torch
    from paper_2106_14402_amd import binding as B
    from paper_2106_14402_amd import spgemm as S
    rng = np.random.default_rng(8)
    A = with_semiring_values(_skewed(3000, 8, 9), "min_plus_i32", rng)
    dU = S.to_device(shuffled(A, rng))
    with pytest.raises(B.SpgError) as e:
        S.spgemm(dU, dU, "min_plus_i32", options=opts(unsorted=-1))
    assert e.value.status == 1
    # a duplicate hidden in an unsorted slice is found on the sorted copy
    U = shuffled(A, rng)
    r = int(np.argmax(np.diff(U.ptr) >= 3))
    lo = int(U.ptr[r])
    idx = U.idx.copy()
    idx[lo + 2] = idx[lo]
    if idx[lo + 1] > idx[lo]:
        idx[lo], idx[lo + 1] = idx[lo + 1], idx[lo]      # keep the slice unsorted
    dD = S.to_device(spgen.SparseMatrix(U.nrows, U.ncols, "csr", U.ptr, idx, U.val))
    with pytest.raises(B.SpgError) as e:
        S.spgemm(dD, S.to_device(A), "min_plus_i32")
    assert e.value.status == 1
    torch.cuda.synchronize()


def test_matrix_check_flags():
    import torch
    from paper_2106_14402_amd import binding as B
    from paper_2106_14402_amd import spgemm as S
    rng = np.random.default_rng(10)
    A = with_semiring_values(_skewed(2000, 8, 11), "min_plus_i32", rng)
    ws = torch.zeros(64, dtype=torch.int32, device="cuda")
    d = S.to_device(A)
    assert B.spg_matrix_check(B.make_matrix(d.nrows, d.ncols, 0, d.ptr, d.idx, d.val), ws) == 0
    u = S.to_device(shuffled(A, rng))
    assert B.spg_matrix_check(B.make_matrix(u.nrows, u.ncols, 0, u.ptr, u.idx, u.val), ws) & 8
    bad = d.idx.clone()
    bad[0] = A.ncols
    assert B.spg_matrix_check(B.make_matrix(d.nrows, d.ncols, 0, d.ptr, bad, d.val), ws) & 4


def test_b_checked_skips_sort_room():
    """b_checked = 1 (a resident operand checked once): no room to sort B, the
    product of sorted operands is unchanged."""
    from paper_2106_14402_amd import spgemm as S
    A = with_semiring_values(_skewed(4000, 8, 12), "min_plus_i32", np.random.default_rng(13))
    dA = S.to_device(A)
    p0 = S.Product(dA, dA, "min_plus_i32")
    p1 = S.Product(dA, dA, "min_plus_i32", opts(b_checked=1))
    assert p1.ws.numel() < p0.ws.numel()
    p0.close()
    p1.close()
    got = run_gpu(A, A, "min_plus_i32", opts(b_checked=1))
    assert_parity(A, A, "min_plus_i32", got)
