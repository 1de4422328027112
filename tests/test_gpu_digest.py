"""The digests of a device result (torch on the GPU) equal the oracle's, so
the full-output comparison of the R-MAT scale-20 square can rely on them."""
import numpy as np
import pytest

import oracle
import spgen
from tests import digest_util as D
from tests.gpu_util import with_semiring_values

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("sr", ["min_plus_i32", "pattern", "max_times_f32"])
def test_device_block_digests_equal_oracle(sr):
    import torch

    from paper_2106_14402_amd import spgemm as S
    code = "or_and_bool" if sr == "pattern" else sr
    A = spgen.rmat_graph(0, 10, np.random.default_rng(8), symmetric=True, n=20000)
    if sr != "pattern":
        A = with_semiring_values(A, sr, np.random.default_rng(9))
    dA = S.to_device(A)
    C = S.spgemm(dA, dA, code)
    torch.cuda.synchronize()
    bn, bh = D.block_digests(C.ptr, C.idx, C.val, A.nrows, block=1024, max_entries=1 << 20)
    on, oh = oracle.block_digests(*oracle.digest(A, A, code), 0, 1024)
    assert np.array_equal(bn, on)
    assert np.array_equal(bh, oh)
