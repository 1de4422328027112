"""MI355X-native local semiring sparse product C = A (x).(+) B.

The hot path of Combinatorial BLAS 2.0's SpGEMM (arXiv 2106.14402, Sec. 4.1)
as hand-written gfx950 kernels behind a C ABI (include/spg.h); this package
is the thin Python binding plus the batched and served front ends.
"""
from .binding import SEMIRINGS, SpgError, load  # noqa: F401

__all__ = ["SEMIRINGS", "SpgError", "load"]
