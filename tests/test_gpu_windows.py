"""Windowed dense symbolic phase: the heavy rows' patterns are computed as
(row, column window) work items taken from per-window queues.  Each product
is compared with the oracle element by element; the windows must give the
row sizes, the rank chunk counts and the kept bitmaps the numeric phase
relies on, for any number of windows, workgroup size and grid."""
import numpy as np
import pytest

import spgen
from tests.gpu_util import assert_parity, run_gpu, with_semiring_values

pytestmark = pytest.mark.gpu


def opts(**kw):
    from paper_2106_14402_amd import binding
    return binding.make_options(**kw)


def _skewed(n, ef, seed, symmetric=False):
    return spgen.rmat_graph(0, ef, np.random.default_rng(seed), symmetric=symmetric, n=n)


MODES = {
    # two windows; fixed panels for the numeric phase (chunks wider than the windows)
    "win2": dict(hash_max_flops=32, hash_max_nnz=32, sym_windows=2),
    # three windows (the last one narrower), rank passes over chunks of 256 columns
    "win3_rank": dict(hash_max_flops=32, hash_max_nnz=32, lds_budget=1024, dense_threads=256, sym_windows=3),
    # eight windows with kept bitmaps written window by window
    "win8_rank_kept": dict(hash_max_flops=32, hash_max_nnz=32, lds_budget=1024, dense_threads=256,
                           bitmap_mib=1, sym_windows=8),
    # 40 windows of 128 columns (more windows than XCDs: every queue is taken by stealing too)
    "win64_kept": dict(hash_max_flops=32, hash_max_nnz=32, bitmap_mib=1, sym_windows=64),
    # one-wave workgroups, two per compute unit
    "win8_small_grid": dict(hash_max_flops=32, hash_max_nnz=32, lds_budget=1024, dense_threads=256,
                            bitmap_mib=1, sym_windows=8, win_threads=64, win_wgs=1),
    # a kept-bitmap budget smaller than the eligible rows: the rest walk B again
    "win4_partly_kept": dict(hash_max_flops=32, hash_max_nnz=32, lds_budget=1024, dense_threads=256,
                             bitmap_mib=1, sym_windows=4),
}


@pytest.mark.parametrize("sr", ["min_plus_i32", "or_and_bool", "plus_times_f64", "max_times_f32"])
@pytest.mark.parametrize("mode", sorted(MODES))
def test_windowed_symbolic_paths(sr, mode):
    n = 5000 if mode != "win4_partly_kept" else 30000
    A = with_semiring_values(_skewed(n, 10, 4), sr, np.random.default_rng(5))
    if sr == "or_and_bool":
        A = A.with_values(None)  # the pattern-only product (kept-bitmap expansion)
    got = run_gpu(A, A, sr, opts(**MODES[mode]))
    assert_parity(A, A, sr, got)


@pytest.mark.parametrize("sr", ["min_plus_i32", "or_and_bool"])
def test_eight_windows_wide_product(sr):
    """150,000 columns in eight windows of 2^15 columns, rank chunks of 2^14
    columns nested in them, kept bitmaps."""
    A = _skewed(150000, 3, 31, symmetric=True)
    A = with_semiring_values(A, sr, np.random.default_rng(32)) if sr != "or_and_bool" else A
    got = run_gpu(A, A, sr, opts(bitmap_mib=256, sym_windows=8))
    assert_parity(A, A, sr, got)


def test_windows_off_matches_on():
    """One bitmap per row (the default) and eight windows give the same
    product, entry for entry."""
    A = with_semiring_values(_skewed(150000, 3, 33, symmetric=True), "min_plus_i32", np.random.default_rng(34))
    on = run_gpu(A, A, "min_plus_i32", opts(bitmap_mib=256, sym_windows=8))
    off = run_gpu(A, A, "min_plus_i32", opts(bitmap_mib=256))
    for x, y in zip(on, off):
        assert np.array_equal(x, y)
