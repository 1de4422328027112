"""The device-side digest used by the full-output parity test, run here on
CPU tensors, equals the oracle's digests (an independent implementation in
C++): mix64 on random words, slice digests of oracle products of every exact
semiring, and block digests with a ragged last block."""
import numpy as np
import pytest

import oracle
import spgen
from tests import digest_util as D
from tests.gpu_util import with_semiring_values


def test_mix64_matches_oracle():
    import torch
    rng = np.random.default_rng(7)
    x = rng.integers(0, 2**63, size=4096, dtype=np.uint64) * np.uint64(2) + rng.integers(0, 2, 4096, dtype=np.uint64)
    got = D.mix64(torch.from_numpy(x.view(np.int64))).numpy().view(np.uint64)
    assert np.array_equal(got, oracle.mix64(x))


@pytest.mark.parametrize("sr", ["min_plus_i32", "or_and_bool", "max_times_f64", "min_plus_f32", "pattern"])
def test_slice_and_block_digests_match_oracle(sr):
    import torch
    A = spgen.rmat_graph(0, 6, np.random.default_rng(3), symmetric=True, n=3000)
    code = "or_and_bool" if sr == "pattern" else sr
    if sr != "pattern":
        A = with_semiring_values(A, sr, np.random.default_rng(4))
    ptr, idx, val = oracle.spgemm(A, A, code)
    want_n, want_h = oracle.digest(A, A, code)
    tp, ti = torch.from_numpy(ptr), torch.from_numpy(idx)
    tv = None if sr == "pattern" else torch.from_numpy(val)
    n, h = D.slice_digests(tp, ti, tv, 0, A.nrows)
    assert np.array_equal(n.numpy(), want_n)
    assert np.array_equal(h.numpy().view(np.uint64), want_h)
    # blocks of 256 slices (the last one ragged), a few blocks per step
    bn, bh = D.block_digests(tp, ti, tv, A.nrows, block=256, max_entries=20000)
    on, oh = oracle.block_digests(want_n, want_h, 0, 256)
    assert np.array_equal(bn, on) and np.array_equal(bh, oh)
    # a single wrong value or id changes the block digest
    if tv is not None and idx.size:
        tv2 = tv.clone()
        tv2[idx.size // 2] = tv2[idx.size // 2] + 1 if tv2.dtype != torch.uint8 else 1 - tv2[idx.size // 2]
        assert not np.array_equal(D.block_digests(tp, ti, tv2, A.nrows, block=256)[1], oh)
    ti2 = ti.clone()
    ti2[0] = ti2[0] + 1 if ti2[0] + 1 < ti2[1] else ti2[0]
    if not torch.equal(ti2, ti):
        assert not np.array_equal(D.block_digests(tp, ti2, tv, A.nrows, block=256)[1], oh)
