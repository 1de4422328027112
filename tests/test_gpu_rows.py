"""Output formed in batches of slices (spg_numeric_rows) on the GPU: after
one symbolic phase, each range of slices is computed into buffers sized for
that range alone, and every range matches the oracle's slices element by
element; exact semirings also match the single-call result bit for bit."""
import numpy as np
import pytest

import spgen
from tests.gpu_util import assert_parity, with_semiring_values

pytestmark = pytest.mark.gpu


def opts(**kw):
    from paper_2106_14402_amd import binding
    return binding.make_options(**kw)


def _skewed(n, ef, seed, layout="csr"):
    return spgen.rmat_graph(0, ef, np.random.default_rng(seed), symmetric=False, n=n, layout=layout)


MODES = {
    "default": None,
    "all_dense": lambda: opts(hash_max_flops=32, hash_max_nnz=32, rank_panels=-1),
    "rank_all": lambda: opts(hash_max_flops=64, hash_max_nnz=64, lds_budget=8192),
    "rank_kept_bitmaps": lambda: opts(hash_max_flops=32, hash_max_nnz=32, lds_budget=1024, dense_threads=256,
                                      bitmap_mib=1),
    "rank_wide": lambda: opts(hash_max_flops=64, hash_max_nnz=64, lds_budget=8192, rank_shapes=2),
    "rank_fixed": lambda: opts(hash_max_flops=32, hash_max_nnz=32, sym_panel_log2=8, lds_budget=1024,
                               rank_dense_div=100000),
}


def _batched(A, sr, options, max_nnz):
    """(full result, [(rb, re, range result)]) as numpy arrays."""
    import torch

    from paper_2106_14402_amd import spgemm as S
    dA = S.to_device(A)
    p = S.Product(dA, dA, sr, options)
    p.symbolic()
    full = p.numeric()
    torch.cuda.synchronize()
    full = (full.ptr.cpu().numpy(), full.idx.cpu().numpy(), None if full.val is None else full.val.cpu().numpy())
    ranges = p.row_batches(max_nnz)
    parts = []
    for rb, re in ranges:
        C = p.numeric_rows(rb, re)
        torch.cuda.synchronize()
        parts.append((rb, re, (C.ptr.cpu().numpy(), C.idx.cpu().numpy(),
                               None if C.val is None else C.val.cpu().numpy())))
    p.close()
    return full, parts


def _check(A, sr, full, parts):
    fp, fi, fv = full
    ns = fp.size - 1
    assert parts[0][0] == 0 and parts[-1][1] == ns
    for rb, re, got in parts:
        assert_parity(A, A, sr, got, select=np.arange(rb, re))
        gp, gi, gv = got
        lo, hi = fp[rb], fp[re]
        assert np.array_equal(gp, fp[rb:re + 1] - lo)
        assert np.array_equal(gi, fi[lo:hi])
        if gv is not None and not sr.startswith("plus_times"):
            assert np.array_equal(gv.view(np.uint8), fv[lo:hi].view(np.uint8))


@pytest.mark.parametrize("sr", ["plus_times_f64", "plus_times_f32", "min_plus_i32", "or_and_bool",
                                "max_times_f32"])
@pytest.mark.parametrize("mode", sorted(MODES))
def test_row_batches_match(sr, mode):
    """R-MAT n=5000: ranges over hash, dense, rank and kept-bitmap rows."""
    A = with_semiring_values(_skewed(5000, 10, 4), sr, np.random.default_rng(5))
    o = MODES[mode]() if MODES[mode] else None
    full, parts = _batched(A, sr, o, max_nnz=40000)
    assert len(parts) > 3
    _check(A, sr, full, parts)


def test_pattern_only_kept_bitmaps():
    A = _skewed(5000, 10, 6)
    full, parts = _batched(A, "or_and_bool", opts(hash_max_flops=32, hash_max_nnz=32, bitmap_mib=64), 30000)
    _check(A, "or_and_bool", full, parts)


@pytest.mark.parametrize("layout", ["csr", "csc"])
def test_ranges_any_order_then_full(layout):
    """Ranges in reverse order, single slices, empty ranges, and a whole
    spg_numeric afterwards (it re-bins the whole product)."""
    import torch

    from paper_2106_14402_amd import spgemm as S
    sr = "min_plus_i32"
    A = with_semiring_values(_skewed(3000, 12, 7, layout), sr, np.random.default_rng(8))
    dA = S.to_device(A)
    p = S.Product(dA, dA, sr)
    p.symbolic()
    ref = p.numeric()
    torch.cuda.synchronize()
    ns = p.nslices
    cuts = [0, 1, 2, 2, 700, 1900, ns - 1, ns]
    for rb, re in reversed(list(zip(cuts[:-1], cuts[1:]))):
        C = p.numeric_rows(rb, re)
        torch.cuda.synchronize()
        lo, hi = int(ref.ptr[rb]), int(ref.ptr[re])
        assert C.nnz == hi - lo
        assert torch.equal(C.idx, ref.idx[lo:hi]) and torch.equal(C.val, ref.val[lo:hi])
        assert torch.equal(C.ptr, ref.ptr[rb:re + 1] - lo)
    again = p.numeric()
    torch.cuda.synchronize()
    assert torch.equal(again.idx, ref.idx) and torch.equal(again.val, ref.val)
    p.close()


def test_errors():
    import torch

    from paper_2106_14402_amd import binding as B_
    from paper_2106_14402_amd import spgemm as S
    A = _skewed(2000, 8, 9)
    A = with_semiring_values(A, "plus_times_f64", np.random.default_rng(1))
    dA = S.to_device(A)
    p = S.Product(dA, dA, "plus_times_f64")
    with pytest.raises(B_.SpgError):  # before the symbolic phase
        B_.spg_numeric_rows(p.plan, p.ws, 0, 1, None, None)
    p.symbolic()
    buf = torch.empty(1, dtype=torch.int32, device="cuda")
    for rb, re in [(-1, 3), (5, 4), (0, 2001)]:
        with pytest.raises(B_.SpgError):
            B_.spg_numeric_rows(p.plan, p.ws, rb, re, buf, buf)
    p.close()
    q = S.Product(dA, dA, "plus_times_f64", opts(hash_max_flops=64, hash_max_nnz=64, split_panels=1,
                                                 lds_budget=4096))
    q.symbolic()
    with pytest.raises(B_.SpgError):  # split work items cover every slice
        q.numeric_rows(0, 100)
    whole = q.numeric_rows(0, q.nslices)  # the whole product is still allowed
    torch.cuda.synchronize()
    assert whole.nnz == q.c_nnz
    q.close()
