"""Batched products on the GPU: every product of a mixed batch against the
oracle and against its own single call, and hipGraph replays of the numeric
phase against the eager run."""
import numpy as np
import pytest

import oracle
import spgen
from tests.gpu_util import assert_parity

pytestmark = pytest.mark.gpu


def _batch(nprod=40, n_lo=256, n_hi=6000, d_lo=4, d_hi=24):
    return spgen.batch_mix(nprod=nprod, n_lo=n_lo, n_hi=n_hi, d_lo=d_lo, d_hi=d_hi)


def _run_batch(items, extra=None, options=None):
    import torch

    from paper_2106_14402_amd import batch as BT
    from paper_2106_14402_amd import spgemm as S
    mats = [S.to_device(it.A) for it in items]
    srs = [it.semiring for it in items]
    As, Bs = list(mats), list(mats)
    if extra:
        for A, Bm, sr in extra:
            As.append(S.to_device(A))
            Bs.append(S.to_device(Bm))
            srs.append(sr)
    bp = BT.BatchProduct(As, Bs, srs, options)
    bp.symbolic()
    bp.numeric()
    torch.cuda.synchronize()
    return bp


def _host(C):
    return (C.ptr.cpu().numpy(), C.idx.cpu().numpy(), None if C.val is None else C.val.cpu().numpy())


def test_mixed_batch_matches_oracle():
    items = _batch()
    rng = np.random.default_rng(3)
    csc = spgen.mcl_matrix(3000, 10.0, 1.0, rng)
    pat = spgen.rmat_graph(0, 8, rng, symmetric=True, n=2500)
    mpf = spgen.erdos_renyi(900, 7, rng, values="f32")
    extra = [(csc, csc, "plus_times_f32"), (pat, pat, "or_and_bool"), (mpf, mpf, "min_plus_f32")]
    bp = _run_batch(items, extra)
    for b, it in enumerate(items):
        assert_parity(it.A, it.A, it.semiring, _host(bp.result(b)))
    for j, (A, Bm, sr) in enumerate(extra):
        assert_parity(A, Bm, sr, _host(bp.result(len(items) + j)))
    bp.close()


def test_batch_equals_single_calls_bit_exact():
    from paper_2106_14402_amd import spgemm as S
    items = [it for it in _batch(24) if it.semiring == "min_plus_i32"]
    bp = _run_batch(items)
    for b, it in enumerate(items):
        dA = S.to_device(it.A)
        C = S.spgemm(dA, dA, it.semiring)
        one = _host(C)
        got = _host(bp.result(b))
        for x, y in zip(one, got):
            assert np.array_equal(x, y)
    bp.close()


def test_forced_dense_and_panels_in_batch():
    items = _batch(16, n_lo=2000, n_hi=9000, d_lo=8, d_hi=20)
    from paper_2106_14402_amd import binding
    o = binding.make_options(hash_max_flops=64, hash_max_nnz=64, lds_budget=8192, dense_threads=256)
    bp = _run_batch(items, options=o)
    for b, it in enumerate(items):
        assert_parity(it.A, it.A, it.semiring, _host(bp.result(b)))
    bp.close()


def test_batched_esc_rows_on_and_off():
    """Rows of low compression ratio take the batched expand-sort-compress
    classes (up to 8192 products); with them off the same rows take the
    hash and dense kernels: both match the oracle, and the exact semirings
    agree entry for entry."""
    from paper_2106_14402_amd import binding
    items = _batch(16, n_lo=2000, n_hi=12000, d_lo=20, d_hi=60)
    on = _run_batch(items)
    off = _run_batch(items, options=binding.make_options(esc_max_flops=-1))
    t_items = [(b, it) for b, it in enumerate(items)]
    for b, it in t_items:
        got = _host(on.result(b))
        assert_parity(it.A, it.A, it.semiring, got)
        if it.semiring == "min_plus_i32":
            for x, y in zip(got, _host(off.result(b))):
                assert np.array_equal(x, y)
    on.close()
    off.close()


def test_graph_replay_matches_eager():
    import torch
    items = _batch(20)
    bp = _run_batch(items)
    eager_idx = bp.c_idx.clone()
    eager_val = bp.c_val.clone()
    bp.capture()
    for rep in range(3):
        bp.c_idx.fill_(-7)
        bp.c_val.fill_(0xAB)
        torch.cuda.synchronize()
        bp.replay()
        torch.cuda.synchronize()
        # eager work between replays
        _ = (torch.arange(1000, device=bp.device) * 2).sum().item()
        assert torch.equal(bp.c_idx, eager_idx), f"replay {rep} ids differ"
        # (+,x) values may differ in the last bits between runs; exact ones may not
        for b, it in enumerate(items):
            got = bp.result(b)
            if it.semiring == "min_plus_i32":
                lo, n = bp.val_off[b], bp.c_nnz[b] * 4
                assert torch.equal(bp.c_val[lo:lo + n], eager_val[lo:lo + n])
            else:
                assert_parity(it.A, it.A, it.semiring, _host(got))
    bp.close()


def test_batch_phase_timings_and_capture():
    """Timed plans report every phase of an eager call; the capture made
    with timing on replays to the eager result (no event inside the graph)."""
    import torch

    from paper_2106_14402_amd import binding
    items = _batch(16, n_lo=2000, n_hi=9000, d_lo=8, d_hi=20)
    o = binding.make_options(hash_max_flops=64, hash_max_nnz=64, timing=1)
    bp = _run_batch(items, options=o)
    t = bp.timings()
    assert set(t) == {"sym_hash", "sym_dense", "num_hash", "num_dense", "num_esc"}
    assert all(v >= 0 for v in t.values()) and t["num_dense"] > 0 and t["sym_dense"] > 0
    eager_idx = bp.c_idx.clone()
    bp.capture()
    for _ in range(2):
        bp.c_idx.fill_(-7)
        torch.cuda.synchronize()
        bp.replay()
        torch.cuda.synchronize()
        assert torch.equal(bp.c_idx, eager_idx)
    for b, it in enumerate(items):
        assert_parity(it.A, it.A, it.semiring, _host(bp.result(b)))
    bp.close()
    untimed = _run_batch(items[:2])
    with pytest.raises(binding.SpgError):
        untimed.timings()
    untimed.close()


def test_empty_and_degenerate_products_in_batch():
    rng = np.random.default_rng(5)
    empty = spgen.from_pairs(30, 30, np.zeros(0, np.int64), np.zeros(0, np.int64), np.zeros(0, np.float64))
    zero_rows = spgen.from_pairs(0, 30, np.zeros(0, np.int64), np.zeros(0, np.int64), np.zeros(0, np.float64))
    F = spgen.erdos_renyi(30, 3, rng, values="f64")
    extra = [(empty, F, "plus_times_f64"), (zero_rows, F, "plus_times_f64"), (F, F, "plus_times_f64")]
    bp = _run_batch([], extra)
    for j, (A, Bm, sr) in enumerate(extra):
        assert_parity(A, Bm, sr, _host(bp.result(j)))
    bp.close()


def test_autotuned_batch_matches_oracle_and_uses_cache(tmp_path):
    """Knobs picked by timing change launch shapes only: every product still
    matches the oracle; a second batch of the same shape reads the cache."""
    from paper_2106_14402_amd import autotune as AT
    from paper_2106_14402_amd import batch as BT
    from paper_2106_14402_amd import spgemm as S
    items = _batch(16, n_hi=3000)
    mats = [S.to_device(it.A) for it in items]
    srs = [it.semiring for it in items]
    cache = str(tmp_path / "tune.json")
    rec = AT.tune_batch(mats, mats, srs, cache, reps=1)
    assert not rec["from_cache"] and rec["ms"] is not None and rec["ms"] <= rec["default_ms"]
    bp = BT.BatchProduct(mats, mats, srs, "auto", autotune_cache=cache)
    assert bp.tuning["from_cache"] and bp.tuning["knobs"] == rec["knobs"]
    bp.symbolic()
    bp.numeric()
    for b, it in enumerate(items):
        assert_parity(it.A, it.A, it.semiring, _host(bp.result(b)))
    bp.close()


@pytest.mark.parametrize("budget", [8192, 65536, 131072])
def test_whole_row_rank_passes_in_batch(budget):
    """Heavy rows of small products take one rank pass over all their
    columns when their entries fit the value slots (more of them with a
    larger LDS budget), else fixed panels; both against the oracle."""
    items = _batch(12, n_lo=3000, n_hi=60000, d_lo=8, d_hi=24)
    from paper_2106_14402_amd import binding
    o = binding.make_options(hash_max_flops=64, hash_max_nnz=64, lds_budget=budget, dense_threads=512)
    bp = _run_batch(items, options=o)
    for b, it in enumerate(items):
        assert_parity(it.A, it.A, it.semiring, _host(bp.result(b)))
    bp.close()
