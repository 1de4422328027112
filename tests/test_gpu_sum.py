"""Semiring sums (the merge of partial products) on the GPU, through the C ABI
(spg_sum_plan_create), against the oracle's sum, and Sparse SUMMA's identity
on the GPU: the sum of the partial products over a split of the inner
dimension equals the whole product."""
import numpy as np
import pytest

import oracle
import spgen
from tests.gpu_util import NP_DTYPE, with_semiring_values
from tests.test_oracle_pins import ALL, VALKIND, random_sparse

pytestmark = pytest.mark.gpu


def _gpu_sum(parts, sr, options=None):
    import torch

    from paper_2106_14402_amd import spgemm as S
    C = S.spg_sum([S.to_device(P) for P in parts], sr, options)
    torch.cuda.synchronize()
    return C.ptr.cpu().numpy(), C.idx.cpu().numpy(), None if C.val is None else C.val.cpu().numpy()


def _abs_sum(parts):
    return oracle.sum_parts([P.with_values(np.abs(P.val.astype(np.float64))) for P in parts], "plus_times_f64")


def _compare(parts, sr, got, want=None):
    gp, gi, gv = got
    op, oi, ov = want if want is not None else oracle.sum_parts(parts, sr)
    assert np.array_equal(gp, op), "slice sizes differ"
    assert np.array_equal(gi, oi), "ids differ"
    if gv is None:
        assert sr == "or_and_bool"
        return
    if sr.startswith("plus_times"):
        _, _, absv = _abs_sum(parts)
        tol = {"plus_times_f64": 1e-12, "plus_times_f32": 1e-5}[sr]
        assert np.all(np.abs(gv.astype(np.float64) - ov) <= tol * absv)
    else:
        assert np.array_equal(gv.view(np.uint8), ov.astype(gv.dtype).view(np.uint8))


@pytest.mark.parametrize("sr", ALL)
@pytest.mark.parametrize("layout", ["csr", "csc"])
@pytest.mark.parametrize("k", [1, 3])
def test_sum_matches_oracle(sr, layout, k):
    rng = np.random.default_rng(50 + k)
    parts = [random_sparse(300, 257, 0.05, rng, VALKIND[sr], layout, signed=True) for _ in range(k)]
    _compare(parts, sr, _gpu_sum(parts, sr))


def test_sum_pattern_only_and_empty_parts():
    rng = np.random.default_rng(7)
    parts = [random_sparse(200, 300, 0.03, rng, "bool").with_values(None) for _ in range(3)]
    parts.append(spgen.SparseMatrix(200, 300, "csr", np.zeros(201, np.int64), np.zeros(0, np.int32), None))
    _compare(parts, "or_and_bool", _gpu_sum(parts, "or_and_bool"))


@pytest.mark.parametrize("sr", ["min_plus_i32", "plus_times_f32", "max_times_f64"])
def test_sum_heavy_rows(sr):
    """Rows whose union exceeds the LDS hash tables (dense and rank paths)."""
    rng = np.random.default_rng(8)
    m, n, k = 40, 120000, 3
    parts = []
    for _ in range(k):
        degs = rng.integers(0, 9000, size=m)
        major, minor = spgen.distinct_minor(m, n, degs, rng)
        P = spgen.from_pairs(m, n, major, minor, None, "csr", presorted=True)
        parts.append(with_semiring_values(P, sr, rng))
    _compare(parts, sr, _gpu_sum(parts, sr))


@pytest.mark.parametrize("sr", ["plus_times_f64", "min_plus_i32", "or_and_bool", "max_times_f32"])
def test_summa_partial_products_on_gpu(sr):
    import torch

    from paper_2106_14402_amd import spgemm as S
    from tests.test_oracle_sum import _col_block, _row_block
    rng = np.random.default_rng(60)
    A = with_semiring_values(spgen.rmat_graph(0, 10, rng, symmetric=False, n=3000), sr, rng)
    cuts = [0, 500, 1400, 2200, 3000]
    partials = []
    for lo, hi in zip(cuts[:-1], cuts[1:]):
        Ab, Bb = S.to_device(_col_block(A, lo, hi)), S.to_device(_row_block(A, lo, hi))
        partials.append(S.spgemm(Ab, Bb, sr))
    C = S.spg_sum(partials, sr)
    full = S.spgemm(S.to_device(A), S.to_device(A), sr)
    torch.cuda.synchronize()
    assert torch.equal(C.ptr, full.ptr) and torch.equal(C.idx, full.idx)
    if C.val is not None:
        if sr == "plus_times_f64":
            want = oracle.spgemm(A, A, sr)
            absv = oracle.spgemm(A.with_values(np.abs(A.val)), A.with_values(np.abs(A.val)), sr)[2]
            assert np.all(np.abs(C.val.cpu().numpy() - want[2]) <= 1e-12 * absv)
        else:
            assert torch.equal(C.val, full.val)
