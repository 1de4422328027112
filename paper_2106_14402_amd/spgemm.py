"""Python front end of the semiring sparse product on one MI355X.

torch supplies device memory and streams; every step of the product runs in
libspg's kernels through the C entry points in ``binding``.
"""
from __future__ import annotations

import dataclasses
from typing import Optional

import numpy as np
import torch

from . import binding as B_

IN_DTYPE = {
    "plus_times_f64": torch.float64, "plus_times_f32": torch.float32, "min_plus_i32": torch.int32,
    "min_plus_f32": torch.float32, "or_and_bool": torch.uint8, "max_times_f64": torch.float64,
    "max_times_f32": torch.float32,
}
OUT_DTYPE = dict(IN_DTYPE)


@dataclasses.dataclass
class DeviceMatrix:
    """Compressed sparse matrix on the device (int64 ptr, int32 idx)."""

    nrows: int
    ncols: int
    layout: str          # "csr" or "csc"
    ptr: torch.Tensor
    idx: torch.Tensor
    val: Optional[torch.Tensor]

    @property
    def nnz(self) -> int:
        return int(self.idx.numel())

    def descriptor(self) -> B_.spg_matrix:
        lay = B_.SPG_CSR if self.layout == "csr" else B_.SPG_CSC
        return B_.make_matrix(self.nrows, self.ncols, lay, self.ptr, self.idx, self.val)


def to_device(M, device="cuda", value_dtype: Optional[torch.dtype] = None) -> DeviceMatrix:
    """Copy a host matrix with numpy ``ptr``/``idx``/``val`` arrays to the device."""
    ptr = torch.from_numpy(M.ptr).to(device=device, dtype=torch.int64)
    idx = torch.from_numpy(M.idx).to(device=device, dtype=torch.int32)
    val = None
    if M.val is not None:
        val = torch.from_numpy(M.val).to(device=device)
        if value_dtype is not None:
            val = val.to(value_dtype)
    return DeviceMatrix(M.nrows, M.ncols, M.layout, ptr, idx, val)


class Product:
    """One product C = A (x).(+) B: plan, workspace, symbolic and numeric."""

    def __init__(self, A: DeviceMatrix, B: DeviceMatrix, semiring: str,
                 options: Optional[B_.spg_options] = None, stream=None):
        self.A, self.B, self.semiring = A, B, semiring
        self.stream = stream if stream is not None else torch.cuda.current_stream(A.ptr.device)
        self._da, self._db = A.descriptor(), B.descriptor()
        self.plan = B_.spg_plan_create(self._da, self._db, semiring, options, self.stream)
        self.ws = torch.empty(max(1, B_.spg_workspace_size(self.plan)), dtype=torch.uint8,
                              device=A.ptr.device)
        if A.layout == "csr":
            self.nslices, self.out_rows, self.out_cols = A.nrows, A.nrows, B.ncols
        else:
            self.nslices, self.out_rows, self.out_cols = B.ncols, A.nrows, B.ncols
        self.c_ptr = None
        self.c_nnz = None

    def symbolic(self, c_ptr: Optional[torch.Tensor] = None) -> int:
        if c_ptr is None:
            c_ptr = torch.empty(self.nslices + 1, dtype=torch.int64, device=self.A.ptr.device)
        self.c_ptr = c_ptr
        self.c_nnz = B_.spg_symbolic(self.plan, self.ws, self.c_ptr)
        return self.c_nnz

    def pattern_only(self) -> bool:
        return self.semiring == "or_and_bool" and self.A.val is None and self.B.val is None

    def numeric(self, c_idx: Optional[torch.Tensor] = None, c_val: Optional[torch.Tensor] = None) -> DeviceMatrix:
        dev = self.A.ptr.device
        if c_idx is None:
            c_idx = torch.empty(self.c_nnz, dtype=torch.int32, device=dev)
        if c_val is None and not self.pattern_only():
            c_val = torch.empty(self.c_nnz, dtype=OUT_DTYPE[self.semiring], device=dev)
        B_.spg_numeric(self.plan, self.ws, c_idx, c_val)
        return DeviceMatrix(self.out_rows, self.out_cols, self.A.layout, self.c_ptr, c_idx, c_val)

    def numeric_rows(self, row_begin: int, row_end: int, c_idx: Optional[torch.Tensor] = None,
                     c_val: Optional[torch.Tensor] = None) -> DeviceMatrix:
        """Output slices [row_begin, row_end) only, into buffers sized for
        that range; returns them as a matrix of row_end - row_begin slices."""
        dev = self.A.ptr.device
        ends = self.c_ptr[[row_begin, row_end]].cpu()
        nnz = int(ends[1] - ends[0])
        if c_idx is None:
            c_idx = torch.empty(nnz, dtype=torch.int32, device=dev)
        if c_val is None and not self.pattern_only():
            c_val = torch.empty(nnz, dtype=OUT_DTYPE[self.semiring], device=dev)
        B_.spg_numeric_rows(self.plan, self.ws, row_begin, row_end, c_idx, c_val)
        ptr = self.c_ptr[row_begin:row_end + 1] - ends[0].to(dev)
        k = row_end - row_begin
        rows, cols = (k, self.out_cols) if self.A.layout == "csr" else (self.out_rows, k)
        return DeviceMatrix(rows, cols, self.A.layout, ptr, c_idx[:nnz], None if c_val is None else c_val[:nnz])

    def row_batches(self, max_nnz: int):
        """Slice ranges whose outputs hold at most max_nnz entries each (a
        slice larger than that gets a range of its own), from c_ptr."""
        return row_batches(self.c_ptr.cpu().numpy(), max_nnz)

    def stats(self):
        return B_.spg_plan_stats(self.plan)

    def options(self):
        """The options the plan runs with (defaults filled in)."""
        return B_.spg_plan_options(self.plan)

    def hash_max_nnz(self) -> int:
        return int(self.options().hash_max_nnz)

    def hash_max_flops(self) -> int:
        return int(self.options().hash_max_flops)

    def rank_dense_div(self) -> int:
        return int(self.options().rank_dense_div)

    def timings(self) -> dict:
        return B_.spg_plan_timings(self.plan)

    def bins(self):
        return B_.spg_plan_bins(self.plan)

    def close(self):
        if self.plan:
            B_.spg_plan_destroy(self.plan)
            self.plan = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def row_batches(c_ptr, max_nnz: int):
    """Greedy split of slices 0..len(c_ptr)-2 into consecutive ranges
    [rb, re) with c_ptr[re] - c_ptr[rb] <= max_nnz, or a single slice when
    that slice alone is larger; every slice is in exactly one range."""
    c_ptr = np.asarray(c_ptr, dtype=np.int64)
    m = c_ptr.size - 1
    if max_nnz < 1:
        raise ValueError("max_nnz must be positive")
    out, rb = [], 0
    while rb < m:
        re = int(np.searchsorted(c_ptr, c_ptr[rb] + max_nnz, side="right")) - 1
        re = min(max(re, rb + 1), m)
        out.append((rb, re))
        rb = re
    return out


def inflate_f32(C: DeviceMatrix, r: float, in_place: bool = True, stream=None) -> DeviceMatrix:
    """Raise every value to the power r and renormalise each slice to sum 1."""
    stream = stream if stream is not None else torch.cuda.current_stream(C.ptr.device)
    out = C.val if in_place else torch.empty_like(C.val)
    B_.spg_inflate_f32(C.descriptor(), r, out, stream)
    return DeviceMatrix(C.nrows, C.ncols, C.layout, C.ptr, C.idx, out)


class SumPlan(Product):
    """C = (+)_t P_t for k parts of one shape, given stacked in one matrix
    (slice i of part t is slice t*m + i); runs through the product engine."""

    def __init__(self, P: DeviceMatrix, k: int, semiring: str, options=None, stream=None):
        self.A, self.B, self.semiring = P, P, semiring
        self.stream = stream if stream is not None else torch.cuda.current_stream(P.ptr.device)
        self._dp = P.descriptor()
        self.plan = B_.spg_sum_plan_create(k, self._dp, semiring, options, self.stream)
        self.ws = torch.empty(max(1, B_.spg_workspace_size(self.plan)), dtype=torch.uint8,
                              device=P.ptr.device)
        major = P.nrows if P.layout == "csr" else P.ncols
        m = major // k
        self.nslices = m
        if P.layout == "csr":
            self.out_rows, self.out_cols = m, P.ncols
        else:
            self.out_rows, self.out_cols = P.nrows, m
        self.c_ptr = None
        self.c_nnz = None


def stack(parts) -> DeviceMatrix:
    """k device matrices of one shape and layout stacked slice-wise."""
    lay = parts[0].layout
    assert all(p.layout == lay and p.nrows == parts[0].nrows and p.ncols == parts[0].ncols for p in parts)
    ptrs, base = [parts[0].ptr[:1]], 0
    for p in parts:
        ptrs.append(p.ptr[1:] + base)
        base += p.nnz
    ptr = torch.cat(ptrs)
    idx = torch.cat([p.idx for p in parts])
    val = None if parts[0].val is None else torch.cat([p.val for p in parts])
    k = len(parts)
    if lay == "csr":
        return DeviceMatrix(parts[0].nrows * k, parts[0].ncols, lay, ptr, idx, val)
    return DeviceMatrix(parts[0].nrows, parts[0].ncols * k, lay, ptr, idx, val)


def spg_sum(parts, semiring: str, options=None, stream=None) -> DeviceMatrix:
    """(+)_t parts[t] over the semiring (the merge of partial products)."""
    P = stack(parts)
    p = SumPlan(P, len(parts), semiring, options, stream)
    try:
        p.symbolic()
        return p.numeric()
    finally:
        p.close()


def spgemm(A: DeviceMatrix, B: DeviceMatrix, semiring: str, options=None, stream=None) -> DeviceMatrix:
    """C = A (x).(+) B; both operands in one layout, C in that layout."""
    p = Product(A, B, semiring, options, stream)
    try:
        p.symbolic()
        return p.numeric()
    finally:
        p.close()


def prune_f32(C: DeviceMatrix, thresh: float, stream=None) -> DeviceMatrix:
    """Keep the entries of a float32 matrix with value >= thresh."""
    stream = stream if stream is not None else torch.cuda.current_stream(C.ptr.device)
    d = C.descriptor()
    dev = C.ptr.device
    ws = torch.empty(max(1, B_.spg_prune_workspace_size(d)), dtype=torch.uint8, device=dev)
    nmajor = C.nrows if C.layout == "csr" else C.ncols
    new_ptr = torch.empty(nmajor + 1, dtype=torch.int64, device=dev)
    nnz = B_.spg_prune_count_f32(d, thresh, ws, new_ptr, stream)
    new_idx = torch.empty(nnz, dtype=torch.int32, device=dev)
    new_val = torch.empty(nnz, dtype=torch.float32, device=dev)
    B_.spg_prune_apply_f32(d, thresh, ws, new_ptr, new_idx, new_val, stream)
    return DeviceMatrix(C.nrows, C.ncols, C.layout, new_ptr, new_idx, new_val)


def select_f32(C: DeviceMatrix, S: int, stream=None) -> DeviceMatrix:
    """Keep at most S entries per slice of a float32 matrix: the largest
    values, ties to the smaller id, in id order."""
    stream = stream if stream is not None else torch.cuda.current_stream(C.ptr.device)
    d = C.descriptor()
    dev = C.ptr.device
    ws = torch.empty(max(1, B_.spg_prune_workspace_size(d)), dtype=torch.uint8, device=dev)
    nmajor = C.nrows if C.layout == "csr" else C.ncols
    new_ptr = torch.empty(nmajor + 1, dtype=torch.int64, device=dev)
    nnz = B_.spg_select_count_f32(d, S, ws, new_ptr, stream)
    new_idx = torch.empty(nnz, dtype=torch.int32, device=dev)
    new_val = torch.empty(nnz, dtype=torch.float32, device=dev)
    B_.spg_select_apply_f32(d, S, ws, new_ptr, new_idx, new_val, stream)
    return DeviceMatrix(C.nrows, C.ncols, C.layout, new_ptr, new_idx, new_val)
