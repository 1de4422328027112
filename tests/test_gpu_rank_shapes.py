"""Rank passes over 2^20 output columns with every pass shape in play: rows
of a few thousand entries spread over all columns (bounded by the bitmap
width: the shape with fewer slots over more chunks) and rows of tens of
thousands (bounded by the slots: the wider-slot shapes).  Compared with the
oracle element by element, and with the five-shape plan entry for entry."""
import numpy as np
import pytest

import spgen
from tests.gpu_util import assert_parity, run_gpu, with_semiring_values

pytestmark = pytest.mark.gpu

NCOLS = 1 << 20


def _operands(sr, seed):
    rng = np.random.default_rng(seed)
    kmid = 40000
    degs = np.concatenate([np.full(600, 250), np.full(120, 1500), rng.integers(0, 40, 200)])
    major, minor = spgen.distinct_minor(degs.size, kmid, degs, rng)
    A = spgen.from_pairs(degs.size, kmid, major, minor, None, presorted=True)
    B = spgen.erdos_renyi(kmid, 30, rng, values=None, ncols=NCOLS)
    return (with_semiring_values(A, sr, np.random.default_rng(seed + 1)),
            with_semiring_values(B, sr, np.random.default_rng(seed + 2)))


@pytest.mark.parametrize("sr", ["min_plus_i32", "plus_times_f64", "max_times_f32"])
def test_all_rank_shapes_over_wide_rows(sr):
    from paper_2106_14402_amd import binding
    A, B = _operands(sr, 71)
    got = run_gpu(A, B, sr)
    assert_parity(A, B, sr, got)
    if sr == "min_plus_i32":
        five = run_gpu(A, B, sr, binding.make_options(rank_shapes=5))
        for x, y in zip(got, five):
            assert np.array_equal(x, y)

