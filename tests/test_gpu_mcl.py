"""Markov-clustering iteration on the GPU: expansion (the product), pruning
and inflation with renormalisation, each against the oracle."""
import numpy as np
import pytest

import oracle
import spgen

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("r", [2.0, 1.5])
@pytest.mark.parametrize("layout", ["csc", "csr"])
@pytest.mark.parametrize("n,mean_deg", [(5000, 40.0), (20000, 150.0)])
def test_inflation_matches_oracle(r, layout, n, mean_deg):
    """Slices of a few dozen entries (held in registers) and of several
    thousand (two passes over the slice)."""
    import torch

    from paper_2106_14402_amd import spgemm as S
    M = spgen.mcl_matrix(n, mean_deg, 1.0, np.random.default_rng(11))
    if mean_deg > 100:
        assert np.diff(M.ptr).max() > 1024
    if layout == "csr":  # the same arrays read as the transpose's rows
        M = spgen.SparseMatrix(M.ncols, M.nrows, "csr", M.ptr, M.idx, M.val)
    d = S.to_device(M)
    out = S.inflate_f32(d, r, in_place=False)
    torch.cuda.synchronize()
    got = out.val.cpu().numpy().astype(np.float64)
    want = oracle.inflate(M, r)
    # float32 powers (a few ulp) and one float32 rounding of the quotient
    assert np.all(np.abs(got - want) <= 1e-6 * want + 1e-12)
    assert torch.equal(d.val.cpu(), torch.from_numpy(M.val))  # input untouched


def test_mcl_iteration():
    """Expansion, prune at 1e-4 and inflation (r=2) of a column-stochastic
    matrix: each step against the oracle on the GPU's own input of that step;
    the result is column-stochastic again."""
    import torch

    from paper_2106_14402_amd import spgemm as S
    M = spgen.mcl_matrix(20000, 30.0, 1.0, np.random.default_rng(12))
    d = S.to_device(M)
    C = S.spgemm(d, d, "plus_times_f32")
    P = S.prune_f32(C, 1e-4)
    I = S.inflate_f32(P, 2.0, in_place=False)
    torch.cuda.synchronize()
    Ph = spgen.SparseMatrix(P.nrows, P.ncols, "csc", P.ptr.cpu().numpy(), P.idx.cpu().numpy(),
                            P.val.cpu().numpy())
    Cv = C.val.cpu().numpy()
    keep = Cv >= np.float32(1e-4)
    assert np.array_equal(Ph.val, Cv[keep])
    want = oracle.inflate(Ph, 2.0)
    got = I.val.cpu().numpy().astype(np.float64)
    assert np.all(np.abs(got - want) <= 1e-6 * want + 1e-12)
    cs = np.concatenate([[0.0], np.cumsum(got)])
    sums = cs[Ph.ptr[1:]] - cs[Ph.ptr[:-1]]
    nonempty = np.diff(Ph.ptr) > 0
    assert np.all(np.abs(sums[nonempty] - 1.0) < 1e-5)


@pytest.mark.parametrize("in_place", [False, True])
def test_inflation_zero_and_empty_slices(in_place):
    """Slices whose values are all zero are left as they are (also into a
    separate output buffer); empty slices stay empty; the others sum to 1."""
    import torch

    from paper_2106_14402_amd import spgemm as S
    ptr = np.array([0, 3, 3, 5, 6, 6], np.int64)
    idx = np.array([0, 2, 5, 1, 4, 3], np.int32)
    val = np.array([0.0, 0.0, 0.0, 1.0, 3.0, 0.0], np.float32)
    M = spgen.SparseMatrix(6, 5, "csc", ptr, idx, val)
    d = S.to_device(M)
    before = d.val.clone()
    out = S.inflate_f32(d, 2.0, in_place=in_place)
    torch.cuda.synchronize()
    got = out.val.cpu().numpy().astype(np.float64)
    want = oracle.inflate(M, 2.0)
    assert np.array_equal(want, [0.0, 0.0, 0.0, 0.1, 0.9, 0.0])
    assert np.all(np.abs(got - want) <= 1e-6 * want)
    if not in_place:
        assert torch.equal(d.val, before)
