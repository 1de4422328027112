"""Selection on the GPU (spg_select_count_f32 / spg_select_apply_f32) equals
the oracle's selection applied to the same float32 input, bit for bit: the
Markov-clustering matrix after expansion and prune, many ties, signed zeros,
long slices (many radix-select passes over thousands of entries), empty
slices, S = 0 and S past every slice."""
import numpy as np
import pytest

import oracle
import spgen

pytestmark = pytest.mark.gpu


def _run(M, S):
    import torch

    from paper_2106_14402_amd import spgemm as Sp
    d = Sp.to_device(M)
    out = Sp.select_f32(d, S)
    torch.cuda.synchronize()
    return out.ptr.cpu().numpy(), out.idx.cpu().numpy(), out.val.cpu().numpy()


def _same(got, M, S):
    want = oracle.select_f32(M.ptr, M.idx, M.val, S)
    assert np.array_equal(got[0], want[0])
    assert np.array_equal(got[1], want[1])
    assert np.array_equal(got[2].view(np.uint32), want[2].view(np.uint32))


def _matrix(lengths, rng, levels=None, layout="csc", nminor=None):
    lengths = np.asarray(lengths, np.int64)
    nminor = nminor or int(max(1, lengths.max()) * 2)
    ptr = np.concatenate([[0], np.cumsum(lengths)]).astype(np.int64)
    idx = np.concatenate([np.sort(rng.choice(nminor, size=int(L), replace=False)) for L in lengths]
                         ).astype(np.int32) if lengths.sum() else np.zeros(0, np.int32)
    if levels is None:
        val = rng.random(idx.size).astype(np.float32)
    else:
        val = np.asarray(levels, np.float32)[rng.integers(0, len(levels), idx.size)]
    if layout == "csc":
        return spgen.SparseMatrix(nminor, lengths.size, "csc", ptr, idx, val)
    return spgen.SparseMatrix(lengths.size, nminor, "csr", ptr, idx, val)


def test_hand_column_and_signed_zeros():
    M = spgen.SparseMatrix(10, 2, "csc", np.array([0, 5, 7], np.int64),
                           np.array([1, 3, 4, 7, 9, 0, 2], np.int32),
                           np.array([0.1, 0.5, 0.2, 0.5, 0.4, -0.0, 0.0], np.float32))
    for S in (0, 1, 2, 3, 5, 6):
        _same(_run(M, S), M, S)
    p, i, v = _run(M, 1)
    assert i.tolist() == [3, 2] and not np.signbit(v[1])


@pytest.mark.parametrize("S", [1, 7, 64, 300, 100000])
def test_mcl_expansion_pruned_then_selected(S):
    """The expansion's own output (prune applied), as the iteration runs it."""
    import torch

    from paper_2106_14402_amd import spgemm as Sp
    A = spgen.config_mcl(n=20000, mean_deg=30.0)
    dA = Sp.to_device(A)
    C = Sp.prune_f32(Sp.spgemm(dA, dA, "plus_times_f32"), 1e-4)
    torch.cuda.synchronize()
    H = spgen.SparseMatrix(C.nrows, C.ncols, "csc", C.ptr.cpu().numpy(), C.idx.cpu().numpy(),
                           C.val.cpu().numpy())
    _same(_run(H, S), H, S)


@pytest.mark.parametrize("layout", ["csc", "csr"])
def test_ties_long_and_empty_slices(layout):
    rng = np.random.default_rng(12)
    lengths = np.concatenate([rng.integers(0, 40, 3000), [0, 0, 1, 255, 256, 257, 9000, 20000, 70000]])
    rng.shuffle(lengths)
    # few distinct values (ties at every cut), with both zeros
    M = _matrix(lengths, rng, levels=[0.25, 0.5, 0.5, 1.0, -0.0, 0.0, 3.0], layout=layout, nminor=200000)
    for S in (1, 10, 256, 5000):
        _same(_run(M, S), M, S)
    M2 = _matrix(lengths, rng, layout=layout, nminor=200000)
    _same(_run(M2, 33), M2, 33)
