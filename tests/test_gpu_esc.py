"""Expand-sort-compress numeric rows (rows whose products are almost all
distinct output entries): forced on and off, every semiring, both layouts,
rows spanning several blocks of A entries, rows with repeated columns
(combined after the sort), and the Markov-clustering product, each compared
with the oracle."""
import numpy as np
import pytest

import spgen
from tests.gpu_util import assert_parity, run_gpu, with_semiring_values

pytestmark = pytest.mark.gpu


def opts(**kw):
    from paper_2106_14402_amd import binding
    return binding.make_options(**kw)


ALL = ["plus_times_f64", "plus_times_f32", "min_plus_i32", "min_plus_f32", "or_and_bool", "max_times_f64",
       "max_times_f32"]


@pytest.mark.parametrize("sr", ALL)
@pytest.mark.parametrize("mode", ["every_row", "default", "off"])
def test_esc_rows_every_semiring(sr, mode):
    """Skewed R-MAT (repeats in most rows): every row up to 4096 products
    through ESC (ratio bound 64), the default choice, and ESC off."""
    A = with_semiring_values(spgen.rmat_graph(0, 8, np.random.default_rng(7), n=3000), sr,
                             np.random.default_rng(8))
    o = {"every_row": opts(esc_ratio_x16=1024), "default": None, "off": opts(esc_max_flops=-1)}[mode]
    got = run_gpu(A, A, sr, o)
    assert_parity(A, A, sr, got)


@pytest.mark.parametrize("sr", ["plus_times_f32", "min_plus_i32", "or_and_bool"])
def test_esc_mcl_csc(sr):
    """Column-stochastic CSC (compression close to 1): most columns take ESC."""
    A = spgen.config_mcl(n=30000, mean_deg=30.0)
    if sr != "plus_times_f32":
        A = with_semiring_values(A, sr, np.random.default_rng(9))
    got = run_gpu(A, A, sr)
    assert_parity(A, A, sr, got)


def test_esc_long_a_rows_and_small_classes():
    """A rows longer than a workgroup's block of entries (several rounds of
    the expansion) and products from 1 to 4096 per row."""
    rng = np.random.default_rng(10)
    n = 20000
    deg = np.concatenate([rng.integers(1, 4, n - 40), rng.integers(1100, 2000, 40)])
    rows = np.repeat(np.arange(n), deg)
    cols = np.concatenate([np.sort(rng.choice(n, size=d, replace=False)) for d in deg])
    A = spgen.SparseMatrix(n, n, "csr", np.concatenate([[0], np.cumsum(deg)]).astype(np.int64),
                           cols.astype(np.int32), rng.random(cols.size))
    _ = rows
    got = run_gpu(A, A, "plus_times_f64", opts(esc_ratio_x16=1024))
    assert_parity(A, A, "plus_times_f64", got)


@pytest.mark.parametrize("sr", ["plus_times_f64", "min_plus_i32", "max_times_f32", "or_and_bool"])
def test_esc_largest_class_among_heavy_rows(sr):
    """Rows of 4097 to 8192 products with almost no repeats (heavy rows of
    the dense symbolic list, over 2^20 columns) take the 8192-product class
    instead of the rank passes; lighter and heavier rows keep their paths."""
    rng = np.random.default_rng(12)
    kmid = 20000
    degs = np.concatenate([rng.integers(60, 110, 1500), rng.integers(1, 40, 300), rng.integers(150, 260, 60)])
    major, minor = spgen.distinct_minor(degs.size, kmid, degs, rng)
    A = spgen.from_pairs(degs.size, kmid, major, minor, None, presorted=True)
    B = spgen.erdos_renyi(kmid, 70, rng, values=None, ncols=1 << 20)
    if sr != "or_and_bool":
        A = with_semiring_values(A, sr, np.random.default_rng(13))
        B = with_semiring_values(B, sr, np.random.default_rng(14))
    got = run_gpu(A, B, sr)
    assert_parity(A, B, sr, got)
    off = run_gpu(A, B, sr, opts(esc_max_flops=4096))
    if sr in ("min_plus_i32", "or_and_bool"):
        for x, y in zip(got, off):
            assert x is None and y is None or np.array_equal(x, y)
