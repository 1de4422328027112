"""Pins of the oracle's inflation step (Markov clustering: values to the
power r, each slice renormalised to sum 1), CPU only."""
import numpy as np

import oracle
import spgen


def _col(vals):
    v = np.asarray(vals, np.float32)
    return spgen.SparseMatrix(len(v), 1, "csc", np.array([0, len(v)], np.int64), np.arange(len(v), dtype=np.int32), v)


def test_worked_example():
    # [1, 2, 3] squared is [1, 4, 9], which sums to 14
    out = oracle.inflate(_col([1.0, 2.0, 3.0]), 2.0)
    assert np.allclose(out, [1 / 14, 4 / 14, 9 / 14], rtol=0, atol=1e-15)


def test_slices_sum_to_one_and_ratios_follow_the_power():
    M = spgen.mcl_matrix(400, 12.0, 1.0, np.random.default_rng(3))
    for r in (1.5, 2.0, 3.0):
        out = oracle.inflate(M, r)
        for s in range(M.ncols):
            lo, hi = M.ptr[s], M.ptr[s + 1]
            assert abs(out[lo:hi].sum() - 1.0) < 1e-12
            if hi - lo >= 2:
                v = M.val[lo:hi].astype(np.float64)
                assert np.allclose(out[lo + 1:hi] / out[lo], (v[1:] / v[0]) ** r, rtol=1e-12)


def test_power_one_keeps_a_stochastic_matrix():
    M = spgen.mcl_matrix(300, 10.0, 1.0, np.random.default_rng(4))
    out = oracle.inflate(M, 1.0)
    # the float32 values already sum to 1 up to their rounding
    assert np.allclose(out, M.val.astype(np.float64), rtol=1e-6)


def test_zero_slice_is_left_alone():
    M = spgen.SparseMatrix(2, 2, "csc", np.array([0, 1, 2], np.int64), np.array([0, 1], np.int32),
                           np.array([0.0, 5.0], np.float32))
    out = oracle.inflate(M, 2.0)
    assert out[0] == 0.0 and out[1] == 1.0
