"""CPU oracle for the local semiring sparse product (test infrastructure).

This package is the plain reference the GPU library is checked against.  Only
``tests/``, the smoke check and the benchmark's CPU-baseline leg may import
it.  It wraps ``oracle.cpp`` (row/column Gustavson with an ordered-map
accumulator, paper Sec. 4.1) through ``ctypes``; it shares no code with the
GPU library.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Optional, Sequence, Tuple

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "oracle.cpp")
LIB = os.path.join(HERE, "liboracle.so")

# Semiring codes (an interface convention, restated here rather than shared).
SEMIRINGS = {
    "plus_times_f64": 0,
    "plus_times_f32": 1,
    "min_plus_i32": 2,
    "min_plus_f32": 3,
    "or_and_bool": 4,
    "max_times_f64": 5,
    "max_times_f32": 6,
}
# Input value dtype and oracle output dtype per semiring.
IN_DTYPE = {0: np.float64, 1: np.float32, 2: np.int32, 3: np.float32, 4: np.uint8, 5: np.float64,
            6: np.float32}
OUT_DTYPE = {0: np.float64, 1: np.float64, 2: np.int32, 3: np.float32, 4: np.uint8, 5: np.float64,
             6: np.float32}

_lib = None


def build(force: bool = True) -> str:
    """Compile ``oracle.cpp`` into ``liboracle.so`` with g++."""
    if force or not os.path.exists(LIB):
        tmp = LIB + ".tmp"
        cmd = ["g++", "-O2", "-std=c++17", "-fopenmp", "-ffp-contract=off", "-fno-fast-math",
               "-fPIC", "-shared", SRC, "-o", tmp]
        subprocess.check_call(cmd)
        os.replace(tmp, LIB)
    return LIB


def load(path: str):
    """Open a compiled oracle library and declare its entry points."""
    L = ctypes.CDLL(path)
    vp, i64, i32 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int
    L.orc_spgemm.restype = vp
    L.orc_spgemm.argtypes = [i32, i32, i64, vp, vp, vp, vp, vp, vp, vp, i32]
    L.orc_sum.restype = vp
    L.orc_sum.argtypes = [i32, i64, i32, vp, vp, vp, i32]
    L.orc_nnz.restype = i64
    L.orc_nnz.argtypes = [vp]
    L.orc_elem_bytes.restype = i32
    L.orc_elem_bytes.argtypes = [vp]
    L.orc_copy.restype = None
    L.orc_copy.argtypes = [vp, vp, vp, vp]
    L.orc_free.restype = None
    L.orc_free.argtypes = [vp]
    L.orc_flops.restype = None
    L.orc_flops.argtypes = [i32, i64, vp, vp, vp, vp, vp, vp]
    L.orc_prune_f32.restype = i64
    L.orc_prune_f32.argtypes = [i64, vp, vp, vp, ctypes.c_float, vp, vp, vp]
    L.orc_digest.restype = i32
    L.orc_digest.argtypes = [i32, i32, i64, vp, vp, vp, vp, vp, vp, vp, i32, vp, vp]
    L.orc_mix64.restype = None
    L.orc_mix64.argtypes = [i64, vp, vp]
    L.orc_select_f32.restype = i64
    L.orc_select_f32.argtypes = [i64, vp, vp, vp, i64, vp, vp, vp]
    return L


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
            build()
        _lib = load(LIB)
    return _lib


def _p(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _code(semiring) -> int:
    return SEMIRINGS[semiring] if isinstance(semiring, str) else int(semiring)


def _arrays(M, code: int, name: str):
    ptr = np.ascontiguousarray(M.ptr, dtype=np.int64)
    idx = np.ascontiguousarray(M.idx, dtype=np.int32)
    val = None
    if M.val is not None:
        val = np.ascontiguousarray(M.val, dtype=IN_DTYPE[code])
    elif code != 4:
        raise ValueError(f"{name}: values are required for semiring {code}")
    return ptr, idx, val


def spgemm(A, B, semiring, select: Optional[Sequence[int]] = None,
           nthreads: int = 0, _lib=None) -> Tuple[np.ndarray, np.ndarray, np.ndarray]:
    """C = A (x).(+) B for the slices ``select`` (rows for CSR, columns for
    CSC; all when None).  A and B are ``spgen.SparseMatrix`` of one layout.
    Returns (ptr, idx, val) of the selected slices, packed in order."""
    code = _code(semiring)
    if A.layout != B.layout:
        raise ValueError("A and B must share a layout")
    if A.ncols != B.nrows:
        raise ValueError("inner dimensions differ")
    layout = 0 if A.layout == "csr" else 1
    nslices = A.nrows if layout == 0 else B.ncols
    Ap, Ai, Av = _arrays(A, code, "A")
    Bp, Bi, Bv = _arrays(B, code, "B")
    sel = None
    if select is not None:
        sel = np.ascontiguousarray(select, dtype=np.int64)
        nsel = sel.size
    else:
        nsel = nslices
    L = _lib or lib()
    h = L.orc_spgemm(code, layout, nsel, _p(sel), _p(Ap), _p(Ai), _p(Av), _p(Bp), _p(Bi), _p(Bv),
                     int(nthreads))
    if not h:
        raise ValueError(f"unknown semiring {semiring}")
    try:
        nnz = L.orc_nnz(h)
        ptr = np.empty(nsel + 1, np.int64)
        idx = np.empty(nnz, np.int32)
        val = np.empty(nnz, OUT_DTYPE[code])
        L.orc_copy(h, _p(ptr), _p(idx), _p(val))
    finally:
        L.orc_free(h)
    return ptr, idx, val


def sum_parts(parts, semiring, nthreads: int = 0, _lib=None) -> Tuple[np.ndarray, np.ndarray, np.ndarray]:
    """(+)_t parts[t] over the semiring, entry by entry (parts: SparseMatrix
    of one shape and layout).  Returns (ptr, idx, val) of the result's slices
    (rows for CSR, columns for CSC)."""
    code = _code(semiring)
    P0 = parts[0]
    if any(p.layout != P0.layout or p.nrows != P0.nrows or p.ncols != P0.ncols for p in parts):
        raise ValueError("parts must share shape and layout")
    m = P0.nrows if P0.layout == "csr" else P0.ncols
    ptrs, idxs, vals, base = [np.zeros(1, np.int64)], [], [], 0
    for p in parts:
        pp, pi, pv = _arrays(p, code, "P")
        ptrs.append(pp[1:] + base)
        idxs.append(pi)
        vals.append(pv)
        base += int(pp[-1])
    Pp = np.ascontiguousarray(np.concatenate(ptrs))
    Pi = np.ascontiguousarray(np.concatenate(idxs) if idxs else np.zeros(0, np.int32))
    Pv = None if vals[0] is None else np.ascontiguousarray(np.concatenate(vals))
    L = _lib or lib()
    h = L.orc_sum(code, m, len(parts), _p(Pp), _p(Pi), _p(Pv), int(nthreads))
    if not h:
        raise ValueError(f"unknown semiring {semiring}")
    try:
        nnz = L.orc_nnz(h)
        ptr = np.empty(m + 1, np.int64)
        idx = np.empty(nnz, np.int32)
        val = np.empty(nnz, OUT_DTYPE[code])
        L.orc_copy(h, _p(ptr), _p(idx), _p(val))
    finally:
        L.orc_free(h)
    return ptr, idx, val


def inflate(C, r: float) -> np.ndarray:
    """Inflation with renormalisation, in float64: every slice's values to
    the power r, divided by their sum (slices summing to 0 are kept).
    Returns the new values in C's entry order."""
    v = np.asarray(C.val, dtype=np.float64) ** float(r)
    out = v.copy()
    for s in range(C.ptr.size - 1):
        lo, hi = int(C.ptr[s]), int(C.ptr[s + 1])
        tot = v[lo:hi].sum()
        if tot != 0.0:
            out[lo:hi] = v[lo:hi] / tot
    return out


def flops(A, B, select: Optional[Sequence[int]] = None) -> np.ndarray:
    """Number of (x) operations per output slice."""
    layout = 0 if A.layout == "csr" else 1
    nslices = A.nrows if layout == 0 else B.ncols
    sel = None if select is None else np.ascontiguousarray(select, dtype=np.int64)
    nsel = nslices if sel is None else sel.size
    out = np.empty(nsel, np.int64)
    Ap = np.ascontiguousarray(A.ptr, np.int64)
    Ai = np.ascontiguousarray(A.idx, np.int32)
    Bp = np.ascontiguousarray(B.ptr, np.int64)
    Bi = np.ascontiguousarray(B.idx, np.int32)
    lib().orc_flops(layout, nsel, _p(sel), _p(Ap), _p(Ai), _p(Bp), _p(Bi), _p(out))
    return out


def prune_f32(ptr: np.ndarray, idx: np.ndarray, val: np.ndarray, thresh: float):
    """Keep entries with value >= thresh.  Returns (ptr, idx, val)."""
    ptr = np.ascontiguousarray(ptr, np.int64)
    idx = np.ascontiguousarray(idx, np.int32)
    val = np.ascontiguousarray(val, np.float32)
    nmajor = ptr.size - 1
    L = lib()
    nnz = L.orc_prune_f32(nmajor, _p(ptr), _p(idx), _p(val), float(thresh), None, None, None)
    nptr = np.empty(nmajor + 1, np.int64)
    nidx = np.empty(nnz, np.int32)
    nval = np.empty(nnz, np.float32)
    L.orc_prune_f32(nmajor, _p(ptr), _p(idx), _p(val), float(thresh), _p(nptr), _p(nidx), _p(nval))
    return nptr, nidx, nval


def digest(A, B, semiring, select: Optional[Sequence[int]] = None, nthreads: int = 0,
           _lib=None) -> Tuple[np.ndarray, np.ndarray]:
    """Per-slice digests of C = A (x).(+) B for the slices ``select`` (all
    when None), without holding C: (nnz int64, hash uint64) per slice, the
    hash being the sum over the slice's entries t (ascending ids) of
    mix64(mix64((t << 32) | id) ^ value bits) modulo 2^64, mix64 the output
    function of SplitMix64.  Exact semirings only."""
    code = _code(semiring)
    if A.layout != B.layout or A.ncols != B.nrows:
        raise ValueError("operands do not conform")
    layout = 0 if A.layout == "csr" else 1
    nslices = A.nrows if layout == 0 else B.ncols
    Ap, Ai, Av = _arrays(A, code, "A")
    Bp, Bi, Bv = _arrays(B, code, "B")
    sel = None if select is None else np.ascontiguousarray(select, dtype=np.int64)
    nsel = nslices if sel is None else sel.size
    nnz = np.empty(nsel, np.int64)
    h = np.empty(nsel, np.uint64)
    L = _lib or lib()
    rc = L.orc_digest(code, layout, nsel, _p(sel), _p(Ap), _p(Ai), _p(Av), _p(Bp), _p(Bi), _p(Bv),
                      int(nthreads), _p(nnz), _p(h))
    if rc != 0:
        raise ValueError(f"digests are defined for the exact semirings only, not {semiring}")
    return nnz, h


def mix64(x: np.ndarray) -> np.ndarray:
    """SplitMix64's output function applied to every element."""
    x = np.ascontiguousarray(x, dtype=np.uint64)
    out = np.empty_like(x)
    lib().orc_mix64(x.size, _p(x), _p(out))
    return out


def block_digests(nnz: np.ndarray, h: np.ndarray, first_slice: int = 0,
                  block: int = 1024) -> Tuple[np.ndarray, np.ndarray]:
    """Digests of consecutive blocks of ``block`` slices from per-slice
    digests: the block's entry count, and the sum modulo 2^64 over its slices
    i (global index first_slice + position) of
    mix64(h_i ^ mix64((i << 32) | nnz_i))."""
    nnz = np.asarray(nnz, np.int64)
    h = np.asarray(h, np.uint64)
    i = np.arange(first_slice, first_slice + nnz.size, dtype=np.uint64)
    r = mix64(h ^ mix64((i << np.uint64(32)) | nnz.astype(np.uint64)))
    nb = -(-nnz.size // block)
    pad = nb * block - nnz.size
    rs = np.concatenate([r, np.zeros(pad, np.uint64)]).reshape(nb, block)
    ns = np.concatenate([nnz, np.zeros(pad, np.int64)]).reshape(nb, block)
    with np.errstate(over="ignore"):
        bh = rs.sum(axis=1, dtype=np.uint64)
    return ns.sum(axis=1), bh


def select_f32(ptr: np.ndarray, idx: np.ndarray, val: np.ndarray, S: int):
    """Selection: every slice keeps its S largest values (ties to the
    smaller id), in id order.  Returns (ptr, idx, val)."""
    ptr = np.ascontiguousarray(ptr, np.int64)
    idx = np.ascontiguousarray(idx, np.int32)
    val = np.ascontiguousarray(val, np.float32)
    nmajor = ptr.size - 1
    L = lib()
    nnz = L.orc_select_f32(nmajor, _p(ptr), _p(idx), _p(val), int(S), None, None, None)
    nptr = np.empty(nmajor + 1, np.int64)
    nidx = np.empty(nnz, np.int32)
    nval = np.empty(nnz, np.float32)
    L.orc_select_f32(nmajor, _p(ptr), _p(idx), _p(val), int(S), _p(nptr), _p(nidx), _p(nval))
    return nptr, nidx, nval
