"""Helpers for GPU parity tests: run the HIP path through the C ABI and
compare it with the oracle element by element."""
import numpy as np

import oracle
import spgen

VALKIND = {"plus_times_f64": "f64", "plus_times_f32": "f32", "min_plus_i32": "i32",
           "min_plus_f32": "f32", "or_and_bool": "bool", "max_times_f64": "f64",
           "max_times_f32": "f32"}
NP_DTYPE = {"plus_times_f64": np.float64, "plus_times_f32": np.float32, "min_plus_i32": np.int32,
            "min_plus_f32": np.float32, "or_and_bool": np.uint8, "max_times_f64": np.float64,
            "max_times_f32": np.float32}
# Tolerance of (+,x) relative to (|A||B|)_ij, against the float64 oracle.
PLUS_TOL = {"plus_times_f64": 1e-12, "plus_times_f32": 1e-5}


def with_semiring_values(M, sr, rng, signed=False):
    """The same pattern with values of the semiring's type."""
    if sr == "or_and_bool" and M.val is None:
        return M
    kind = VALKIND[sr]
    if kind == "i32":
        v = rng.integers(1, 256, size=M.nnz).astype(np.int32)
        if signed:
            v = rng.integers(-300, 300, size=M.nnz).astype(np.int32)
    elif kind == "bool":
        v = np.ones(M.nnz, np.uint8)
    else:
        v = rng.random(M.nnz).astype(NP_DTYPE[sr])
        if signed:
            v = (v - 0.5).astype(NP_DTYPE[sr])
    return M.with_values(v)


def run_gpu(A, B, sr, options=None, device="cuda"):
    """C through libspg; returns numpy (ptr, idx, val or None)."""
    import torch

    from paper_2106_14402_amd import spgemm as S

    dA = S.to_device(A, device)
    dB = S.to_device(B, device)
    C = S.spgemm(dA, dB, sr, options=options)
    torch.cuda.synchronize()
    return (C.ptr.cpu().numpy(), C.idx.cpu().numpy(),
            None if C.val is None else C.val.cpu().numpy())


def abs_product(A, B, select=None):
    """(|A||B|)_ij in float64 through the oracle, for tolerance scaling."""
    Aa = A.with_values(np.abs(A.val.astype(np.float64)))
    Ba = B.with_values(np.abs(B.val.astype(np.float64)))
    return oracle.spgemm(Aa, Ba, "plus_times_f64", select=select)


def assert_parity(A, B, sr, got, select=None, want=None):
    """Element-by-element check of a GPU result (or the selected slices of
    it, packed in order) against the oracle."""
    gp, gi, gv = got
    op, oi, ov = want if want is not None else oracle.spgemm(A, B, sr, select=select)
    assert gp.shape == op.shape, "slice count differs"
    assert np.array_equal(gp - gp[0], op), "slice sizes differ"
    assert np.array_equal(gi, oi), "column ids differ"
    if gv is None:
        assert sr == "or_and_bool" and np.all(ov == 1)
        return
    if sr in PLUS_TOL:
        _, _, absv = abs_product(A, B, select)
        err = np.abs(gv.astype(np.float64) - ov)
        bound = PLUS_TOL[sr] * absv
        bad = err > bound
        assert not bad.any(), f"{bad.sum()} values outside tolerance; worst {np.max(err - bound)}"
        if (A.val >= 0).all() and (B.val >= 0).all():
            # non-negative operands: (|A||B|)_ij is C_ij itself, so the bound
            # above is the plain relative error |c - c*| / |c*|
            rel = err <= PLUS_TOL[sr] * np.abs(ov) * (1 + 1e-9) + 1e-300
            assert rel.all(), f"{(~rel).sum()} values over the relative tolerance"
    else:
        assert gv.dtype == ov.dtype
        assert np.array_equal(gv.view(np.uint8), ov.view(np.uint8)), "values differ"


def slices_of(ptr, idx, val, rows):
    """Pack the given slices of a full result in order."""
    rows = np.asarray(rows, dtype=np.int64)
    cnt = ptr[rows + 1] - ptr[rows]
    nptr = np.zeros(rows.size + 1, np.int64)
    np.cumsum(cnt, out=nptr[1:])
    sel = np.concatenate([np.arange(ptr[r], ptr[r + 1]) for r in rows]) if rows.size else np.zeros(0, np.int64)
    return nptr, idx[sel], None if val is None else val[sel]
