"""Batched semiring products: many uneven C_b = A_b (x).(+) B_b at once.

The library bins the rows of every product together and runs one launch per
accumulator class and semiring over all of them; the numeric phase can be
captured into a hipGraph and replayed.  torch only supplies the pooled
device buffers.
"""
from __future__ import annotations

from typing import List, Optional, Sequence

import torch

from . import binding as B_
from .spgemm import OUT_DTYPE, DeviceMatrix

VAL_BYTES = {"plus_times_f64": 8, "plus_times_f32": 4, "min_plus_i32": 4, "min_plus_f32": 4,
             "or_and_bool": 1, "max_times_f64": 8, "max_times_f32": 4}


class BatchProduct:
    """options: None (library defaults), an spg_options, or "auto": knob
    values from the autotuner (timed on this batch the first time a batch of
    its shape is seen on this device, then read from autotune_cache)."""

    def __init__(self, As: Sequence[DeviceMatrix], Bs: Sequence[DeviceMatrix], semirings: Sequence[str],
                 options=None, stream=None, autotune_cache: Optional[str] = None):
        assert len(As) == len(Bs) == len(semirings)
        self.tuning = None
        if isinstance(options, str):
            if options != "auto":
                raise ValueError(f"options must be None, spg_options or 'auto', not {options!r}")
            from . import autotune
            self.tuning = autotune.tune_batch(As, Bs, semirings,
                                              autotune_cache if autotune_cache else autotune.DEFAULT_CACHE)
            options = autotune.make_options(self.tuning["knobs"])
        self.As, self.Bs, self.semirings = list(As), list(Bs), list(semirings)
        self.n = len(As)
        self.device = As[0].ptr.device if As else torch.device("cuda")
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self._da = [a.descriptor() for a in As]
        self._db = [b.descriptor() for b in Bs]
        self.plan = B_.spg_batch_plan_create(self._da, self._db, self.semirings, options, self.stream)
        self.ws = torch.empty(max(256, B_.spg_batch_workspace_size(self.plan)), dtype=torch.uint8,
                              device=self.device)
        self.nslices = [a.nrows if a.layout == "csr" else b.ncols for a, b in zip(As, Bs)]
        self.pool_off = [0]
        for m in self.nslices:
            self.pool_off.append(self.pool_off[-1] + m + 1)
        self.c_ptr = torch.empty(max(1, self.pool_off[-1]), dtype=torch.int64, device=self.device)
        self.c_nnz = self.idx_off = self.val_off = None
        self.c_idx = self.c_val = None

    def symbolic(self):
        self.c_nnz, self.idx_off, self.val_off = B_.spg_batch_symbolic(self.plan, self.ws, self.c_ptr, self.n)
        return self.c_nnz

    def allocate(self):
        self.c_idx = torch.empty(max(1, self.idx_off[-1]), dtype=torch.int32, device=self.device)
        self.c_val = torch.empty(max(8, self.val_off[-1]), dtype=torch.uint8, device=self.device)

    def numeric(self):
        if self.c_idx is None:
            self.allocate()
        B_.spg_batch_numeric(self.plan, self.ws, self.c_idx, self.c_val, self.val_off)

    def capture(self):
        if self.c_idx is None:
            self.allocate()
        B_.spg_batch_graph_capture(self.plan, self.ws, self.c_idx, self.c_val, self.val_off)

    def replay(self):
        B_.spg_batch_graph_launch(self.plan)

    def stats(self):
        return B_.spg_batch_stats(self.plan)

    def timings(self) -> dict:
        """Phase times (ms) of the last eager call; needs options.timing."""
        return B_.spg_batch_timings(self.plan)

    def result(self, b: int) -> DeviceMatrix:
        """Views of product b's output inside the pools."""
        sr = self.semirings[b]
        ptr = self.c_ptr[self.pool_off[b]:self.pool_off[b + 1]]
        nnz = self.c_nnz[b]
        idx = self.c_idx[self.idx_off[b]:self.idx_off[b] + nnz]
        pattern = sr == "or_and_bool" and self.As[b].val is None and self.Bs[b].val is None
        val = None
        if not pattern:
            vb = VAL_BYTES[sr]
            raw = self.c_val[self.val_off[b]:self.val_off[b] + nnz * vb]
            val = raw.view(OUT_DTYPE[sr]) if nnz > 0 else torch.empty(0, dtype=OUT_DTYPE[sr], device=self.device)
        A, Bm = self.As[b], self.Bs[b]
        return DeviceMatrix(A.nrows, Bm.ncols, A.layout, ptr, idx, val)

    def close(self):
        if self.plan:
            B_.spg_batch_plan_destroy(self.plan)
            self.plan = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
