"""ctypes binding of libspg (include/spg.h), argument marshalling only.

Every function keeps its C name.  Device buffers are torch tensors on a ROCm
device; their data pointers cross the boundary as plain addresses, and the
stream is the raw hipStream_t of a torch stream.  Nothing here computes any
part of the product: when the library is missing, loading raises.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libspg.so")

SPG_CSR, SPG_CSC = 0, 1
# scratch of spg_prune_count_f32_noalloc (int64 words) and the slices it serves
SPG_NOALLOC_SCRATCH_WORDS = 8192
SPG_NOALLOC_MAX_SLICES = (SPG_NOALLOC_SCRATCH_WORDS - 1) * 8192
SEMIRINGS = {
    "plus_times_f64": 0,
    "plus_times_f32": 1,
    "min_plus_i32": 2,
    "min_plus_f32": 3,
    "or_and_bool": 4,
    "max_times_f64": 5,
    "max_times_f32": 6,
}
STATUS = {
    0: "SPG_OK", 1: "SPG_E_INVALID", 2: "SPG_E_SHAPE", 3: "SPG_E_LAYOUT", 4: "SPG_E_SEMIRING",
    5: "SPG_E_NOMEM", 6: "SPG_E_OVERFLOW", 7: "SPG_E_DEVICE", 8: "SPG_E_STATE",
}


class SpgError(RuntimeError):
    def __init__(self, status: int, where: str):
        self.status = status
        super().__init__(f"{where}: {STATUS.get(status, status)} ({spg_status_str(status)})")


class spg_matrix(ctypes.Structure):
    _fields_ = [
        ("nrows", ctypes.c_int32),
        ("ncols", ctypes.c_int32),
        ("nnz", ctypes.c_int64),
        ("layout", ctypes.c_int),
        ("ptr", ctypes.c_void_p),
        ("idx", ctypes.c_void_p),
        ("val", ctypes.c_void_p),
    ]


class spg_options(ctypes.Structure):
    _fields_ = [
        ("validate", ctypes.c_int32),
        ("hash_max_flops", ctypes.c_int32),
        ("hash_max_nnz", ctypes.c_int32),
        ("short_seg", ctypes.c_int32),
        ("dense_threads", ctypes.c_int32),
        ("sym_panel_log2", ctypes.c_int32),
        ("lds_budget", ctypes.c_int32),
        ("timing", ctypes.c_int32),
        ("split_panels", ctypes.c_int32),
        ("bitmap_mib", ctypes.c_int32),
        ("seg_mib", ctypes.c_int32),
        ("rank_panels", ctypes.c_int32),
        ("rank_dense_div", ctypes.c_int32),
        ("rank_shapes", ctypes.c_int32),
        ("unsorted", ctypes.c_int32),
        ("b_checked", ctypes.c_int32),
        ("sym_windows", ctypes.c_int32),
        ("win_threads", ctypes.c_int32),
        ("win_wgs", ctypes.c_int32),
        ("pack_b", ctypes.c_int32),
        ("esc_max_flops", ctypes.c_int32),
        ("esc_ratio_x16", ctypes.c_int32),
    ]


_lib = None


def load(path: str = LIB_PATH):
    """Open libspg.so and declare its entry points."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} is missing: build it with paper_2106_14402_amd.build.build()")
    # The HIP runtime torch ships must be the one this library binds to: with
    # the library loaded first, torch would bring a second runtime and the
    # streams it hands over would not be valid here.
    import torch  # noqa: F401
    L = ctypes.CDLL(path)
    vp, i64, st = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int
    pm = ctypes.POINTER(spg_matrix)
    po = ctypes.POINTER(spg_options)
    L.spg_status_str.restype = ctypes.c_char_p
    L.spg_status_str.argtypes = [st]
    L.spg_plan_create.restype = st
    L.spg_plan_create.argtypes = [pm, pm, ctypes.c_int, po, vp, ctypes.POINTER(vp)]
    L.spg_workspace_size.restype = st
    L.spg_workspace_size.argtypes = [vp, ctypes.POINTER(ctypes.c_size_t)]
    L.spg_symbolic.restype = st
    L.spg_symbolic.argtypes = [vp, vp, vp, ctypes.POINTER(i64)]
    L.spg_numeric.restype = st
    L.spg_numeric.argtypes = [vp, vp, vp, vp]
    L.spg_numeric_rows.restype = st
    L.spg_numeric_rows.argtypes = [vp, vp, i64, i64, vp, vp]
    L.spg_plan_stats.restype = st
    L.spg_plan_stats.argtypes = [vp, ctypes.POINTER(i64), ctypes.POINTER(i64)]
    L.spg_plan_timings.restype = st
    L.spg_plan_timings.argtypes = [vp, ctypes.POINTER(ctypes.c_float)]
    L.spg_plan_bins.restype = st
    L.spg_plan_bins.argtypes = [vp, ctypes.POINTER(i64), ctypes.POINTER(i64)]
    L.spg_plan_destroy.restype = st
    L.spg_plan_destroy.argtypes = [vp]
    pint = ctypes.POINTER(ctypes.c_int)
    L.spg_plan_panels.restype = st
    L.spg_plan_panels.argtypes = [vp, pint, pint, pint, pint]
    L.spg_inflate_f32.restype = st
    L.spg_inflate_f32.argtypes = [pm, ctypes.c_float, vp, vp]
    L.spg_sum_plan_create.restype = st
    L.spg_sum_plan_create.argtypes = [ctypes.c_int, pm, ctypes.c_int, po, vp, ctypes.POINTER(vp)]
    L.spg_plan_options.restype = st
    L.spg_plan_options.argtypes = [vp, ctypes.POINTER(spg_options)]
    L.spg_panel_index_size.restype = st
    L.spg_panel_index_size.argtypes = [pm, ctypes.c_int, ctypes.POINTER(ctypes.c_size_t)]
    L.spg_panel_index_build.restype = st
    L.spg_panel_index_build.argtypes = [pm, ctypes.c_int, vp, vp]
    L.spg_plan_set_panels.restype = st
    L.spg_plan_set_panels.argtypes = [vp, ctypes.c_int, vp, ctypes.c_int]
    L.spg_matrix_check.restype = st
    L.spg_matrix_check.argtypes = [pm, vp, vp, ctypes.POINTER(ctypes.c_int)]
    L.spg_prune_workspace_size.restype = st
    L.spg_prune_workspace_size.argtypes = [pm, ctypes.POINTER(ctypes.c_size_t)]
    L.spg_prune_count_f32.restype = st
    L.spg_prune_count_f32.argtypes = [pm, ctypes.c_float, vp, vp, vp, ctypes.POINTER(i64)]
    L.spg_prune_apply_f32.restype = st
    L.spg_prune_apply_f32.argtypes = [pm, ctypes.c_float, vp, vp, vp, vp, vp]
    L.spg_select_count_f32.restype = st
    L.spg_select_count_f32.argtypes = [pm, i64, vp, vp, vp, ctypes.POINTER(i64)]
    L.spg_select_apply_f32.restype = st
    L.spg_select_apply_f32.argtypes = [pm, i64, vp, vp, vp, vp, vp]
    L.spg_prune_count_f32_noalloc.restype = st
    L.spg_prune_count_f32_noalloc.argtypes = [pm, ctypes.c_float, vp, vp, ctypes.POINTER(i64)]
    _declare_batch(L)
    _lib = L
    return L


def _declare_batch(L):
    """Declare the batched entry points."""
    vp, i64, st = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int
    pm = ctypes.POINTER(spg_matrix)
    po = ctypes.POINTER(spg_options)
    pi64 = ctypes.POINTER(i64)
    L.spg_batch_plan_create.restype = st
    L.spg_batch_plan_create.argtypes = [ctypes.c_int, pm, pm, ctypes.POINTER(ctypes.c_int), po, vp,
                                        ctypes.POINTER(vp)]
    L.spg_batch_workspace_size.restype = st
    L.spg_batch_workspace_size.argtypes = [vp, ctypes.POINTER(ctypes.c_size_t)]
    L.spg_batch_symbolic.restype = st
    L.spg_batch_symbolic.argtypes = [vp, vp, vp, pi64, pi64, pi64]
    L.spg_batch_numeric.restype = st
    L.spg_batch_numeric.argtypes = [vp, vp, vp, vp, pi64]
    L.spg_batch_graph_capture.restype = st
    L.spg_batch_graph_capture.argtypes = [vp, vp, vp, vp, pi64]
    L.spg_batch_graph_launch.restype = st
    L.spg_batch_graph_launch.argtypes = [vp]
    L.spg_batch_stats.restype = st
    L.spg_batch_stats.argtypes = [vp, pi64, pi64]
    L.spg_batch_timings.restype = st
    L.spg_batch_timings.argtypes = [vp, ctypes.POINTER(ctypes.c_float)]
    L.spg_batch_plan_destroy.restype = st
    L.spg_batch_plan_destroy.argtypes = [vp]


def _check(status: int, where: str):
    if status != 0:
        raise SpgError(status, where)


def _addr(t) -> Optional[int]:
    if t is None:
        return None
    p = t.data_ptr()
    return p if p else None


def _stream(stream) -> Optional[int]:
    if stream is None:
        import torch
        stream = torch.cuda.current_stream()
    return getattr(stream, "cuda_stream", stream) or None


def make_matrix(nrows: int, ncols: int, layout: int, ptr, idx, val) -> spg_matrix:
    """Descriptor of device arrays (torch tensors); val may be None."""
    nnz = int(idx.numel()) if idx is not None else 0
    return spg_matrix(int(nrows), int(ncols), nnz, int(layout), _addr(ptr), _addr(idx), _addr(val))


def make_options(**kw) -> spg_options:
    o = spg_options()
    for k, v in kw.items():
        setattr(o, k, int(v))
    return o


# ---- the C entry points, one Python function each --------------------------
def spg_status_str(status: int) -> str:
    return load().spg_status_str(int(status)).decode()


def spg_plan_create(A: spg_matrix, B: spg_matrix, semiring, options: Optional[spg_options] = None,
                    stream=None) -> ctypes.c_void_p:
    code = SEMIRINGS[semiring] if isinstance(semiring, str) else int(semiring)
    plan = ctypes.c_void_p()
    _check(load().spg_plan_create(ctypes.byref(A), ctypes.byref(B), code,
                                  ctypes.byref(options) if options is not None else None,
                                  _stream(stream), ctypes.byref(plan)), "spg_plan_create")
    return plan


def spg_inflate_f32(C: spg_matrix, r: float, val_out, stream=None) -> None:
    _check(load().spg_inflate_f32(ctypes.byref(C), float(r), _addr(val_out), _stream(stream)), "spg_inflate_f32")


def spg_sum_plan_create(k: int, P: spg_matrix, semiring, options: Optional[spg_options] = None,
                        stream=None) -> ctypes.c_void_p:
    code = SEMIRINGS[semiring] if isinstance(semiring, str) else int(semiring)
    plan = ctypes.c_void_p()
    _check(load().spg_sum_plan_create(int(k), ctypes.byref(P), code,
                                      ctypes.byref(options) if options is not None else None,
                                      _stream(stream), ctypes.byref(plan)), "spg_sum_plan_create")
    return plan


def spg_workspace_size(plan) -> int:
    n = ctypes.c_size_t()
    _check(load().spg_workspace_size(plan, ctypes.byref(n)), "spg_workspace_size")
    return int(n.value)


def spg_symbolic(plan, ws, c_ptr) -> int:
    nnz = ctypes.c_int64()
    _check(load().spg_symbolic(plan, _addr(ws), _addr(c_ptr), ctypes.byref(nnz)), "spg_symbolic")
    return int(nnz.value)


def spg_numeric(plan, ws, c_idx, c_val) -> None:
    _check(load().spg_numeric(plan, _addr(ws), _addr(c_idx), _addr(c_val)), "spg_numeric")


def spg_numeric_rows(plan, ws, row_begin: int, row_end: int, c_idx, c_val) -> None:
    _check(load().spg_numeric_rows(plan, _addr(ws), int(row_begin), int(row_end), _addr(c_idx), _addr(c_val)),
           "spg_numeric_rows")


def spg_plan_stats(plan):
    f, n = ctypes.c_int64(), ctypes.c_int64()
    _check(load().spg_plan_stats(plan, ctypes.byref(f), ctypes.byref(n)), "spg_plan_stats")
    return int(f.value), int(n.value)


PHASES = ["validate", "flops_bin", "sym_hash", "sym_dense", "scan", "num_hash", "num_dense",
          "sym_panels", "num_panels", "num_expand", "seg_count", "seg_write", "num_rank", "num_esc"]


def spg_plan_timings(plan) -> dict:
    ms = (ctypes.c_float * len(PHASES))()
    _check(load().spg_plan_timings(plan, ms), "spg_plan_timings")
    return {name: float(ms[i]) for i, name in enumerate(PHASES)}


def spg_plan_bins(plan):
    sym = (ctypes.c_int64 * 64)()
    num = (ctypes.c_int64 * 64)()
    _check(load().spg_plan_bins(plan, sym, num), "spg_plan_bins")
    return list(sym), list(num)


def spg_plan_destroy(plan) -> None:
    if plan:
        load().spg_plan_destroy(plan)


def spg_plan_options(plan) -> spg_options:
    """The options the plan runs with, defaults filled in."""
    o = spg_options()
    _check(load().spg_plan_options(plan, ctypes.byref(o)), "spg_plan_options")
    return o


def spg_plan_panels(plan):
    """(sym_wlog2, sym_P, num_wlog2, num_P)"""
    v = [ctypes.c_int() for _ in range(4)]
    _check(load().spg_plan_panels(plan, *[ctypes.byref(x) for x in v]), "spg_plan_panels")
    return tuple(int(x.value) for x in v)


def spg_panel_index_size(R: spg_matrix, wlog2: int) -> int:
    n = ctypes.c_size_t()
    _check(load().spg_panel_index_size(ctypes.byref(R), int(wlog2), ctypes.byref(n)), "spg_panel_index_size")
    return int(n.value)


def spg_panel_index_build(R: spg_matrix, wlog2: int, out, stream=None) -> None:
    _check(load().spg_panel_index_build(ctypes.byref(R), int(wlog2), _addr(out), _stream(stream)),
           "spg_panel_index_build")


def spg_plan_set_panels(plan, which: int, pidx, wlog2: int) -> None:
    _check(load().spg_plan_set_panels(plan, int(which), _addr(pidx), int(wlog2)), "spg_plan_set_panels")


def spg_matrix_check(M: spg_matrix, ws, stream=None) -> int:
    """Error bits of the device check of M (0: well formed and sorted);
    ws: device scratch of at least 256 bytes."""
    flags = ctypes.c_int()
    st = load().spg_matrix_check(ctypes.byref(M), _addr(ws), _stream(stream), ctypes.byref(flags))
    if st not in (0, 1):
        _check(st, "spg_matrix_check")
    return int(flags.value)


def spg_prune_workspace_size(C: spg_matrix) -> int:
    n = ctypes.c_size_t()
    _check(load().spg_prune_workspace_size(ctypes.byref(C), ctypes.byref(n)), "spg_prune_workspace_size")
    return int(n.value)


def spg_prune_count_f32(C: spg_matrix, thresh: float, ws, new_ptr, stream=None) -> int:
    nnz = ctypes.c_int64()
    _check(load().spg_prune_count_f32(ctypes.byref(C), float(thresh), _addr(ws), _stream(stream),
                                      _addr(new_ptr), ctypes.byref(nnz)), "spg_prune_count_f32")
    return int(nnz.value)


def spg_prune_count_f32_noalloc(C: spg_matrix, thresh: float, new_ptr, stream=None) -> int:
    nnz = ctypes.c_int64()
    _check(load().spg_prune_count_f32_noalloc(ctypes.byref(C), float(thresh), _stream(stream), _addr(new_ptr),
                                              ctypes.byref(nnz)), "spg_prune_count_f32_noalloc")
    return int(nnz.value)


def spg_select_count_f32(C: spg_matrix, S: int, ws, new_ptr, stream=None) -> int:
    nnz = ctypes.c_int64()
    _check(load().spg_select_count_f32(ctypes.byref(C), int(S), _addr(ws), _stream(stream), _addr(new_ptr),
                                       ctypes.byref(nnz)), "spg_select_count_f32")
    return int(nnz.value)


def spg_select_apply_f32(C: spg_matrix, S: int, ws, new_ptr, new_idx, new_val, stream=None) -> None:
    _check(load().spg_select_apply_f32(ctypes.byref(C), int(S), _addr(ws), _stream(stream), _addr(new_ptr),
                                       _addr(new_idx), _addr(new_val)), "spg_select_apply_f32")


def spg_prune_apply_f32(C: spg_matrix, thresh: float, ws, new_ptr, new_idx, new_val, stream=None) -> None:
    _check(load().spg_prune_apply_f32(ctypes.byref(C), float(thresh), _addr(ws), _stream(stream),
                                      _addr(new_ptr), _addr(new_idx), _addr(new_val)),
           "spg_prune_apply_f32")


# ---- batched entry points ---------------------------------------------------
def spg_batch_plan_create(As, Bs, semirings, options: Optional[spg_options] = None, stream=None):
    n = len(As)
    arrA = (spg_matrix * max(1, n))(*As)
    arrB = (spg_matrix * max(1, n))(*Bs)
    codes = (ctypes.c_int * max(1, n))(*[SEMIRINGS[x] if isinstance(x, str) else int(x) for x in semirings])
    plan = ctypes.c_void_p()
    _check(load().spg_batch_plan_create(n, arrA, arrB, codes,
                                        ctypes.byref(options) if options is not None else None,
                                        _stream(stream), ctypes.byref(plan)), "spg_batch_plan_create")
    return plan


def spg_batch_workspace_size(plan) -> int:
    n = ctypes.c_size_t()
    _check(load().spg_batch_workspace_size(plan, ctypes.byref(n)), "spg_batch_workspace_size")
    return int(n.value)


def spg_batch_symbolic(plan, ws, c_ptr_pool, nprod: int):
    """Returns (c_nnz[nprod], idx_off[nprod+1], val_off[nprod+1]) as lists."""
    nnz = (ctypes.c_int64 * max(1, nprod))()
    io = (ctypes.c_int64 * (nprod + 1))()
    vo = (ctypes.c_int64 * (nprod + 1))()
    _check(load().spg_batch_symbolic(plan, _addr(ws), _addr(c_ptr_pool), nnz, io, vo), "spg_batch_symbolic")
    return list(nnz)[:nprod], list(io), list(vo)


def _i64_array(values):
    return (ctypes.c_int64 * max(1, len(values)))(*values)


def spg_batch_numeric(plan, ws, c_idx, c_val, val_off) -> None:
    _check(load().spg_batch_numeric(plan, _addr(ws), _addr(c_idx), _addr(c_val), _i64_array(val_off)),
           "spg_batch_numeric")


def spg_batch_graph_capture(plan, ws, c_idx, c_val, val_off) -> None:
    _check(load().spg_batch_graph_capture(plan, _addr(ws), _addr(c_idx), _addr(c_val), _i64_array(val_off)),
           "spg_batch_graph_capture")


def spg_batch_graph_launch(plan) -> None:
    _check(load().spg_batch_graph_launch(plan), "spg_batch_graph_launch")


def spg_batch_stats(plan):
    f, r = ctypes.c_int64(), ctypes.c_int64()
    _check(load().spg_batch_stats(plan, ctypes.byref(f), ctypes.byref(r)), "spg_batch_stats")
    return int(f.value), int(r.value)


BATCH_PHASES = ["sym_hash", "sym_dense", "num_hash", "num_dense", "num_esc"]


def spg_batch_timings(plan) -> dict:
    ms = (ctypes.c_float * len(BATCH_PHASES))()
    _check(load().spg_batch_timings(plan, ms), "spg_batch_timings")
    return {name: float(ms[i]) for i, name in enumerate(BATCH_PHASES)}


def spg_batch_plan_destroy(plan) -> None:
    if plan:
        load().spg_batch_plan_destroy(plan)
