"""The prune count without allocation (its scan partials in the library's own
device array) gives the same offsets and kept count as the count with a
caller workspace, on consecutive calls of decreasing size (the array keeps
the previous call's contents), and oversized inputs are refused before any
device work."""
import numpy as np
import pytest

import spgen

pytestmark = pytest.mark.gpu

THRESH = 1e-4


def _matrix(nslices, seed, layout="csc"):
    """Slices of 0..40 entries, float32 values around the threshold."""
    rng = np.random.default_rng(seed)
    deg = rng.integers(0, 41, size=nslices)
    ptr = np.concatenate([[0], np.cumsum(deg)]).astype(np.int64)
    nnz = int(ptr[-1])
    idx = (np.arange(nnz) - np.repeat(ptr[:-1], deg)).astype(np.int32)
    val = (rng.random(nnz) * 2e-4).astype(np.float32)
    val[rng.random(nnz) < 0.01] = np.float32(THRESH)  # boundary values are kept
    if layout == "csr":
        return spgen.SparseMatrix(nslices, 41, "csr", ptr, idx, val)
    return spgen.SparseMatrix(41, nslices, "csc", ptr, idx, val)


def _both(M):
    import torch

    from paper_2106_14402_amd import binding as B
    from paper_2106_14402_amd import spgemm as S

    d = S.to_device(M, "cuda")
    desc = d.descriptor()
    n = M.ptr.size - 1
    ws = torch.empty(max(1, B.spg_prune_workspace_size(desc)), dtype=torch.uint8, device="cuda")
    ref_ptr = torch.full((n + 1,), -1, dtype=torch.int64, device="cuda")
    ref_nnz = B.spg_prune_count_f32(desc, THRESH, ws, ref_ptr)
    got_ptr = torch.full((n + 1,), -7, dtype=torch.int64, device="cuda")
    got_nnz = B.spg_prune_count_f32_noalloc(desc, THRESH, got_ptr)
    torch.cuda.synchronize()
    return d, desc, (ref_nnz, ref_ptr.cpu().numpy()), (got_nnz, got_ptr.cpu().numpy())


def _expected(M):
    keep = (M.val >= np.float32(THRESH)).astype(np.int64)
    per = np.add.reduceat(keep, M.ptr[:-1]) if M.nnz else np.zeros(M.ptr.size - 1, np.int64)
    per[np.diff(M.ptr) == 0] = 0
    return np.concatenate([[0], np.cumsum(per)])


def test_noalloc_matches_workspace_count_on_shrinking_calls():
    import torch

    from paper_2106_14402_amd import binding as B

    # 300,000 slices (37 scan tiles), then 20,000 (3 tiles, ragged), then 8,192
    # (exactly one tile) and a CSR matrix of 1 slice
    for nslices, seed, layout in ((300_000, 1, "csc"), (20_000, 2, "csc"), (8192, 3, "csc"), (1, 4, "csr")):
        M = _matrix(nslices, seed, layout)
        d, desc, (rn, rp), (gn, gp) = _both(M)
        want = _expected(M)
        assert rn == gn == int(want[-1]), (nslices, rn, gn, int(want[-1]))
        assert np.array_equal(rp, gp) and np.array_equal(gp, want), nslices
        # the apply phase takes the offsets of the no-allocation count
        new_ptr = torch.from_numpy(gp).to("cuda")
        new_idx = torch.empty(max(1, gn), dtype=torch.int32, device="cuda")
        new_val = torch.empty(max(1, gn), dtype=torch.float32, device="cuda")
        B.spg_prune_apply_f32(desc, THRESH, None, new_ptr, new_idx, new_val)
        torch.cuda.synchronize()
        kept = M.val >= np.float32(THRESH)
        assert np.array_equal(new_idx.cpu().numpy()[:gn], M.idx[kept])
        assert np.array_equal(new_val.cpu().numpy()[:gn], M.val[kept])


def test_noalloc_refuses_more_slices_than_its_scratch_serves():
    """Refused on the host, before the scratch is looked up or a kernel runs:
    the descriptor's arrays are never read."""
    import ctypes

    import torch

    from paper_2106_14402_amd import binding as B

    n = B.SPG_NOALLOC_MAX_SLICES + 1
    tiny = torch.zeros(4, dtype=torch.int64, device="cuda")
    desc = B.spg_matrix(4, n, 0, B.SPG_CSC, tiny.data_ptr(), tiny.data_ptr(), tiny.data_ptr())
    nnz = ctypes.c_int64(-1)
    st = B.load().spg_prune_count_f32_noalloc(ctypes.byref(desc), ctypes.c_float(THRESH), None,
                                               ctypes.c_void_p(tiny.data_ptr()), ctypes.byref(nnz))
    assert st == 5  # SPG_E_NOMEM
    assert nnz.value == -1
