"""GPU parity: the HIP path through the C ABI against the oracle, element by
element, on seeded inputs that span every accumulator (LDS hash classes,
dense bitmap, dense value panels with one and many panels), both layouts,
every semiring and the degenerate cases."""
import numpy as np
import pytest

import oracle
import spgen
from tests.gpu_util import assert_parity, run_gpu, with_semiring_values

pytestmark = pytest.mark.gpu

ALL = list(oracle.SEMIRINGS)


def opts(**kw):
    from paper_2106_14402_amd import binding
    return binding.make_options(**kw)


def _skewed(n, ef, seed, symmetric=False):
    return spgen.rmat_graph(0, ef, np.random.default_rng(seed), symmetric=symmetric, n=n)


@pytest.mark.parametrize("sr", ALL)
def test_er_config_all_semirings(sr):
    """Erdos-Renyi n=4096, 8 per row (the small workload), every semiring."""
    A = spgen.config_er()
    if sr != "plus_times_f64":
        A = with_semiring_values(A, sr, np.random.default_rng(1))
    got = run_gpu(A, A, sr)
    assert_parity(A, A, sr, got)


@pytest.mark.parametrize("sr", ALL)
def test_skewed_rmat_default_bins(sr):
    """R-MAT n=6000: rows in many hash classes and in the dense path."""
    A = with_semiring_values(_skewed(6000, 12, 2), sr, np.random.default_rng(3))
    got = run_gpu(A, A, sr)
    assert_parity(A, A, sr, got)


@pytest.mark.parametrize("sr", ["plus_times_f64", "min_plus_i32", "or_and_bool", "max_times_f32"])
@pytest.mark.parametrize("mode", ["all_dense", "many_panels", "many_panels_in_sequence",
                                  "many_panels_rewalk", "windows", "all_hash_small_threads",
                                  "rank_small_slots", "rank_all", "rank_kept_bitmaps",
                                  "rank_fixed_via_chunks", "rank_wide", "rank_wide_kept", "rank_narrow_only"])
def test_forced_paths(sr, mode):
    """The same product through forced accumulators: every row dense; dense
    with many narrow panels (panel index in use), as (row, panel) pieces or
    panel after panel in one workgroup; short segments split; rank-compressed
    passes with few value slots (rows over several passes, by slot count and
    by bitmap width), passes with twice the slots for the densest rows, and
    fixed panels taken over the chunk index."""
    A = with_semiring_values(_skewed(5000, 10, 4), sr, np.random.default_rng(5))
    o = {"all_dense": opts(hash_max_flops=32, hash_max_nnz=32),
         "many_panels": opts(hash_max_flops=32, hash_max_nnz=32, sym_panel_log2=8, lds_budget=1024,
                             dense_threads=256, split_panels=1),
         "many_panels_in_sequence": opts(hash_max_flops=32, hash_max_nnz=32, sym_panel_log2=8,
                                         lds_budget=1024, dense_threads=256, split_panels=-1,
                                         rank_panels=-1),
         # 128 value slots per pass, chunks of 128 columns, bitmap of 64 chunks
         "rank_small_slots": opts(hash_max_flops=32, hash_max_nnz=32, sym_panel_log2=8, lds_budget=1024,
                                  dense_threads=256),
         "rank_all": opts(hash_max_flops=64, hash_max_nnz=64, lds_budget=8192, rank_dense_div=1),
         "rank_kept_bitmaps": opts(hash_max_flops=32, hash_max_nnz=32, lds_budget=1024, dense_threads=256,
                                   bitmap_mib=1),
         # rows at least 1/4 dense take passes with twice the slots
         "rank_wide": opts(hash_max_flops=64, hash_max_nnz=64, lds_budget=8192, rank_shapes=2),
         "rank_wide_kept": opts(hash_max_flops=32, hash_max_nnz=32, lds_budget=1024, dense_threads=256,
                                bitmap_mib=1, rank_shapes=3),
         "rank_narrow_only": opts(hash_max_flops=64, hash_max_nnz=64, lds_budget=8192, rank_shapes=1),
         "rank_fixed_via_chunks": opts(hash_max_flops=32, hash_max_nnz=32, sym_panel_log2=8, lds_budget=1024,
                                       rank_dense_div=100000),
         # no room for segment lists: pieces re-walk their rows
         "many_panels_rewalk": opts(hash_max_flops=32, hash_max_nnz=32, sym_panel_log2=8, lds_budget=1024,
                                    dense_threads=256, seg_mib=1, split_panels=1),
         "windows": opts(hash_max_flops=64, hash_max_nnz=512, lds_budget=4096, split_panels=1),
         "all_hash_small_threads": opts(short_seg=1, dense_threads=64)}[mode]
    got = run_gpu(A, A, sr, o)
    assert_parity(A, A, sr, got)


@pytest.mark.parametrize("sr", ["plus_times_f64", "plus_times_f32", "min_plus_i32", "max_times_f64",
                                "or_and_bool"])
@pytest.mark.parametrize("div,mib", [(4, 0), (1, 0), (100000, 0), (4, 1), (1, 64)])
def test_rank_panels_default_widths(sr, div, mib):
    """More columns than one value panel holds (70,000), default slot and chunk
    widths (2^14 columns for 4-byte accumulators, 2^13 for 8-byte; fixed
    panels of two chunks): heavy rows by rank passes, by fixed panels, or a
    mix split by density; pattern walked again or read from kept symbolic
    bitmaps (room for some rows, or for all)."""
    A = with_semiring_values(_skewed(70000, 2, 21, symmetric=True), sr, np.random.default_rng(22))
    got = run_gpu(A, A, sr, opts(rank_dense_div=div, bitmap_mib=mib))
    assert_parity(A, A, sr, got)


def test_pattern_only_bool_null_values():
    A = _skewed(7000, 14, 6)
    assert A.val is None
    got = run_gpu(A, A, "or_and_bool")
    assert got[2] is None
    assert_parity(A, A, "or_and_bool", got)


@pytest.mark.parametrize("mib", [1, 64])
def test_pattern_only_kept_bitmaps(mib):
    """Heavy rows expanded from bitmaps kept by the symbolic phase (a small
    budget keeps only some of them; the rest are recomputed)."""
    A = _skewed(7000, 14, 6)
    got = run_gpu(A, A, "or_and_bool", opts(bitmap_mib=mib, hash_max_flops=64))
    assert_parity(A, A, "or_and_bool", got)


def test_pattern_only_kept_bitmaps_wide():
    """Kept bitmaps wider than one expansion slab (600,000 columns = 18,750
    words, more than the 16,384 words a slab holds): the second slab is read
    while the first is expanded; rows of uneven lengths put the outputs at
    every alignment."""
    rng = np.random.default_rng(21)
    m, n, k = 160, 3000, 600000
    A = spgen.from_pairs(m, n, *spgen.distinct_minor(m, n, rng.integers(40, 160, size=m), rng), None,
                         "csr", presorted=True)
    B = spgen.from_pairs(n, k, *spgen.distinct_minor(n, k, rng.integers(150, 450, size=n), rng), None,
                         "csr", presorted=True)
    got = run_gpu(A, B, "or_and_bool", opts(bitmap_mib=64, hash_max_flops=64))
    assert_parity(A, B, "or_and_bool", got)


def test_bool_one_side_null():
    rng = np.random.default_rng(7)
    A = _skewed(3000, 8, 7)
    Av = A.with_values(rng.integers(0, 2, size=A.nnz).astype(np.uint8))
    got = run_gpu(Av, A, "or_and_bool")
    assert_parity(Av, A, "or_and_bool", got)


@pytest.mark.parametrize("sr", ["plus_times_f32", "min_plus_f32", "or_and_bool", "max_times_f64"])
def test_csc_layout(sr):
    rng = np.random.default_rng(8)
    A = spgen.mcl_matrix(5000, 20.0, 1.0, rng)  # CSC
    A = with_semiring_values(A, sr, rng) if sr != "plus_times_f32" else A
    got = run_gpu(A, A, sr)
    assert_parity(A, A, sr, got)


@pytest.mark.parametrize("sr", ["plus_times_f64", "min_plus_i32"])
def test_rectangular_and_signed(sr):
    rng = np.random.default_rng(9)
    A = spgen.erdos_renyi(700, 9, rng, values=None, ncols=1300)
    major = np.repeat(np.arange(1300), 40)
    minor = rng.integers(0, 2100, size=major.size)
    key = np.unique(major * 2100 + minor)
    B = spgen.from_pairs(1300, 2100, key // 2100, key % 2100, None)
    A = with_semiring_values(A, sr, rng, signed=True)
    B = with_semiring_values(B, sr, rng, signed=True)
    got = run_gpu(A, B, sr)
    assert_parity(A, B, sr, got)


def test_hash_bin_thresholds():
    """Rows whose flops sit at every hash class bound, -1 and +1."""
    rng = np.random.default_rng(10)
    n = 20000
    flops_targets = []
    for c in range(1, 11):
        b = 32 << (c - 1)
        flops_targets += [b - 1, b, b + 1]
    # B: row k has exactly one entry per row... build A rows of single k with deg(B(k,:)) = target
    rows_b, cols_b = [], []
    for k, f in enumerate(flops_targets):
        cols = rng.choice(n, size=min(f, n), replace=False)
        rows_b += [k] * cols.size
        cols_b += cols.tolist()
    B = spgen.from_pairs(n, n, np.array(rows_b), np.array(cols_b), None)
    A = spgen.from_pairs(len(flops_targets), n, np.arange(len(flops_targets)), np.arange(len(flops_targets)), None)
    for sr in ("min_plus_i32", "plus_times_f64"):
        Av, Bv = with_semiring_values(A, sr, rng), with_semiring_values(B, sr, rng)
        assert_parity(Av, Bv, sr, run_gpu(Av, Bv, sr))


def test_degenerate_shapes():
    rng = np.random.default_rng(11)
    empty = lambda m, n: spgen.from_pairs(m, n, np.zeros(0, np.int64), np.zeros(0, np.int64),
                                          np.zeros(0, np.float64))
    F = with_semiring_values(spgen.erdos_renyi(30, 3, rng, values=None), "plus_times_f64", rng)
    for A, B in [(empty(30, 30), F), (F, empty(30, 30)), (empty(0, 30), F), (F, empty(30, 0)),
                 (empty(0, 0), empty(0, 0))]:
        got = run_gpu(A, B, "plus_times_f64")
        assert_parity(A, B, "plus_times_f64", got)
    one = spgen.from_pairs(1, 1, np.array([0]), np.array([0]), np.array([2.5]))
    assert_parity(one, one, "plus_times_f64", run_gpu(one, one, "plus_times_f64"))


def test_dense_row_and_hub_column():
    """One fully dense row of length n and one hub column hit by every row."""
    rng = np.random.default_rng(12)
    n = 9000
    rows, cols = [np.zeros(n, np.int64)], [np.arange(n)]
    rows.append(np.arange(1, n))
    cols.append(np.full(n - 1, 17))
    extra = rng.integers(0, n, size=(n, 3))
    rows.append(np.repeat(np.arange(n), 3))
    cols.append(extra.ravel())
    r = np.concatenate(rows)
    c = np.concatenate(cols)
    key = np.unique(r * n + c)
    A = spgen.from_pairs(n, n, key // n, key % n, None)
    for sr in ("min_plus_i32", "max_times_f64", "or_and_bool"):
        Av = with_semiring_values(A, sr, rng) if sr != "or_and_bool" else A
        assert_parity(Av, Av, sr, run_gpu(Av, Av, sr))


def test_explicit_identity_values_are_structural():
    rng = np.random.default_rng(13)
    A = _skewed(2000, 6, 14)
    v = np.zeros(A.nnz, np.float64)                      # every product is 0 = (+)-identity
    Av = A.with_values(v)
    got = run_gpu(Av, Av, "plus_times_f64")
    assert_parity(Av, Av, "plus_times_f64", got)
    vb = np.zeros(A.nnz, np.uint8)                       # all false: entries stay, values false
    Ab = A.with_values(vb)
    got = run_gpu(Ab, Ab, "or_and_bool")
    assert_parity(Ab, Ab, "or_and_bool", got)
    assert np.all(got[2] == 0)
    big = np.iinfo(np.int32).max
    vi = np.full(A.nnz, big - 1, np.int32)               # saturates to INT32_MAX
    Ai = A.with_values(vi)
    assert_parity(Ai, Ai, "min_plus_i32", run_gpu(Ai, Ai, "min_plus_i32"))


def test_signed_zero_and_denormals():
    rng = np.random.default_rng(15)
    A = _skewed(3000, 8, 16)
    tiny = np.float32(1e-40)                              # float32 denormal
    choices = np.array([0.0, -0.0, tiny, -tiny, 1.0, -1.0], np.float32)
    v = choices[rng.integers(0, choices.size, size=A.nnz)]
    Av = A.with_values(v)
    for sr in ("min_plus_f32", "max_times_f32"):
        assert_parity(Av, Av, sr, run_gpu(Av, Av, sr))


def test_exact_semirings_are_deterministic():
    A = with_semiring_values(_skewed(6000, 12, 17), "min_plus_i32", np.random.default_rng(18))
    g1 = run_gpu(A, A, "min_plus_i32")
    g2 = run_gpu(A, A, "min_plus_i32")
    for x, y in zip(g1, g2):
        assert np.array_equal(x, y)


def test_prune_matches_reprune_and_oracle():
    import torch

    from paper_2106_14402_amd import spgemm as S
    rng = np.random.default_rng(19)
    A = spgen.mcl_matrix(6000, 24.0, 1.0, rng)
    dA = S.to_device(A)
    C = S.spgemm(dA, dA, "plus_times_f32")
    P = S.prune_f32(C, 1e-4)
    torch.cuda.synchronize()
    cp, ci, cv = C.ptr.cpu().numpy(), C.idx.cpu().numpy(), C.val.cpu().numpy()
    # exact: the prune of the GPU's own values
    wp, wi, wv = oracle.prune_f32(cp, ci, cv, 1e-4)
    assert np.array_equal(P.ptr.cpu().numpy(), wp)
    assert np.array_equal(P.idx.cpu().numpy(), wi)
    assert np.array_equal(P.val.cpu().numpy(), wv)
    # against the float64 oracle: presence may differ only inside the band
    op, oi, ov = oracle.spgemm(A, A, "plus_times_f32")
    keep64 = ov >= 1e-4
    keep32 = cv >= np.float32(1e-4)
    assert np.array_equal(ci, oi)
    flips = keep64 != keep32
    assert np.all(np.abs(ov[flips] - 1e-4) <= 1e-5 * ov[flips])


def test_error_codes():
    import torch

    from paper_2106_14402_amd import binding as B
    from paper_2106_14402_amd import spgemm as S
    rng = np.random.default_rng(20)
    A = with_semiring_values(spgen.erdos_renyi(50, 4, rng, values=None), "min_plus_i32", rng)
    dA = S.to_device(A)
    R = S.to_device(spgen.erdos_renyi(40, 4, rng, values="i32"))
    with pytest.raises(B.SpgError) as e:
        S.spgemm(dA, R, "min_plus_i32")                  # 50x50 times 40x40
    assert e.value.status == 2
    Ac = S.DeviceMatrix(50, 50, "csc", dA.ptr, dA.idx, dA.val)
    with pytest.raises(B.SpgError) as e:
        S.spgemm(dA, Ac, "min_plus_i32")
    assert e.value.status == 3
    with pytest.raises(B.SpgError) as e:
        S.spgemm(dA, S.DeviceMatrix(50, 50, "csr", dA.ptr, dA.idx, None), "min_plus_i32")
    assert e.value.status == 4
    bad_idx = dA.idx.clone()
    bad_idx[5] = 50                                       # out of range
    with pytest.raises(B.SpgError) as e:
        S.spgemm(S.DeviceMatrix(50, 50, "csr", dA.ptr, bad_idx, dA.val), dA, "min_plus_i32",
                 options=opts(validate=1))
    assert e.value.status == 1
    uns = dA.idx.clone()
    uns[0], uns[1] = dA.idx[1], dA.idx[0]                 # unsorted row: rejected only without sort room
    with pytest.raises(B.SpgError) as e:
        S.spgemm(S.DeviceMatrix(50, 50, "csr", dA.ptr, uns, dA.val), dA, "min_plus_i32",
                 options=opts(unsorted=-1))
    assert e.value.status == 1
    dup = dA.idx.clone()
    dup[1] = dA.idx[0]                                    # duplicate id in a row
    with pytest.raises(B.SpgError) as e:
        S.spgemm(S.DeviceMatrix(50, 50, "csr", dA.ptr, dup, dA.val), dA, "min_plus_i32")
    assert e.value.status == 1
    bad_ptr = dA.ptr.clone()
    bad_ptr[3] = bad_ptr[4] + 1                           # decreasing offsets
    with pytest.raises(B.SpgError) as e:
        S.spgemm(dA, S.DeviceMatrix(50, 50, "csr", bad_ptr, dA.idx, dA.val), "min_plus_i32")
    assert e.value.status == 1
    p = S.Product(dA, dA, "min_plus_i32")
    with pytest.raises(B.SpgError) as e:
        B.spg_numeric(p.plan, p.ws, None, None)          # numeric before symbolic
    assert e.value.status == 8
    p.close()
    C = S.spgemm(dA, dA, "min_plus_i32", options=opts(validate=1))  # valid input passes validation
    torch.cuda.synchronize()
    assert C.nnz > 0


@pytest.mark.parametrize("case", ["packed_at_limit", "pairs_past_limit", "pairs_negative", "pairs_forced"])
def test_rank_passes_packed_words_and_pairs(case):
    """(min,+) int32 rank passes read B through one 32-bit word per entry
    when every value fits beside the column id (5000 columns: 13 id bits,
    values below 2^19), else through 8-byte pairs; both give the oracle's
    product."""
    rng = np.random.default_rng(41)
    A = _skewed(5000, 10, 4)
    v = rng.integers(0, 1 << 19, size=A.nnz).astype(np.int32)
    if case == "packed_at_limit":
        v[rng.integers(0, A.nnz, 20)] = (1 << 19) - 1
    elif case == "pairs_past_limit":
        v[rng.integers(0, A.nnz, 3)] = 1 << 19
    elif case == "pairs_negative":
        v[rng.integers(0, A.nnz, 3)] = -5
    A = A.with_values(v)
    o = dict(hash_max_flops=32, hash_max_nnz=32, lds_budget=1024, dense_threads=256, bitmap_mib=1)
    if case == "pairs_forced":
        o["pack_b"] = -1
    got = run_gpu(A, A, "min_plus_i32", opts(**o))
    assert_parity(A, A, "min_plus_i32", got)
