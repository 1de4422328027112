"""Host logic of output batching: the split of output slices into ranges
whose entries fit a budget, from the offsets of a symbolic phase."""
import numpy as np
import pytest
from hypothesis import given, settings
from hypothesis import strategies as st

from paper_2106_14402_amd.spgemm import row_batches


def _valid(c_ptr, max_nnz, ranges):
    m = len(c_ptr) - 1
    if m == 0:
        return ranges == []
    assert ranges[0][0] == 0 and ranges[-1][1] == m
    for (a, b), (c, _) in zip(ranges[:-1], ranges[1:]):
        assert b == c
    for rb, re in ranges:
        assert re > rb
        nnz = c_ptr[re] - c_ptr[rb]
        assert nnz <= max_nnz or re == rb + 1
        # greedy: the next slice would not have fit
        if re < m:
            assert c_ptr[re + 1] - c_ptr[rb] > max_nnz
    return True


@settings(max_examples=200, deadline=None)
@given(st.lists(st.integers(0, 50), max_size=60), st.integers(1, 120))
def test_row_batches_cover_and_fit(sizes, max_nnz):
    c_ptr = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    assert _valid(c_ptr, max_nnz, row_batches(c_ptr, max_nnz))


def test_row_batches_examples():
    c_ptr = np.array([0, 3, 3, 10, 11, 30, 31])
    assert row_batches(c_ptr, 10) == [(0, 3), (3, 4), (4, 5), (5, 6)]
    assert row_batches(c_ptr, 1000) == [(0, 6)]
    assert row_batches(np.array([0]), 5) == []
    with pytest.raises(ValueError):
        row_batches(c_ptr, 0)
