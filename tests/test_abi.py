"""The C-ABI library loads and exports every entry point its headers declare
(CPU only: no compute calls), and the host-side binning rules are sound."""
import ctypes
import glob
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_2106_14402_amd", "libspg.so")


def declared_functions():
    names = set()
    for h in glob.glob(os.path.join(ROOT, "include", "*.h")):
        text = open(h).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        for m in re.finditer(r"\b(spg_\w+)\s*\(", text):
            names.add(m.group(1))
    return sorted(names)


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        from paper_2106_14402_amd import build
        build.build()
    return ctypes.CDLL(LIB)


def test_header_declares_entry_points():
    names = declared_functions()
    for must in ("spg_plan_create", "spg_workspace_size", "spg_symbolic", "spg_numeric",
                 "spg_plan_destroy", "spg_status_str", "spg_prune_count_f32", "spg_prune_apply_f32"):
        assert must in names


def test_every_declared_symbol_is_exported(lib):
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, f"not exported: {missing}"


def test_status_strings(lib):
    lib.spg_status_str.restype = ctypes.c_char_p
    for code in range(9):
        assert lib.spg_status_str(code)


def test_plan_create_rejects_bad_descriptors_without_gpu(lib):
    """Host-only validation paths (no device work is launched)."""
    from paper_2106_14402_amd import binding as B

    B.load(LIB)
    dummy = ctypes.c_void_p(0x1000)  # never dereferenced by plan creation
    A = B.spg_matrix(4, 5, 3, B.SPG_CSR, dummy.value, dummy.value, dummy.value)
    Bm = B.spg_matrix(6, 4, 3, B.SPG_CSR, dummy.value, dummy.value, dummy.value)
    plan = ctypes.c_void_p()
    L = B.load()
    assert L.spg_plan_create(ctypes.byref(A), ctypes.byref(Bm), 0, None, None, ctypes.byref(plan)) == 2
    Bm = B.spg_matrix(5, 4, 3, B.SPG_CSC, dummy.value, dummy.value, dummy.value)
    assert L.spg_plan_create(ctypes.byref(A), ctypes.byref(Bm), 0, None, None, ctypes.byref(plan)) == 3
    Bm = B.spg_matrix(5, 4, 3, B.SPG_CSR, dummy.value, dummy.value, None)
    assert L.spg_plan_create(ctypes.byref(A), ctypes.byref(Bm), 0, None, None, ctypes.byref(plan)) == 4
    assert L.spg_plan_create(ctypes.byref(A), ctypes.byref(Bm), 9, None, None, ctypes.byref(plan)) == 4
    # OR-AND accepts missing values (pattern only); a valid plan is host-only
    assert L.spg_plan_create(ctypes.byref(A), ctypes.byref(Bm), 4, None, None, ctypes.byref(plan)) == 0
    n = ctypes.c_size_t()
    assert L.spg_workspace_size(plan, ctypes.byref(n)) == 0 and n.value > 0
    # numeric before symbolic
    assert L.spg_numeric(plan, None, None, None) == 8
    assert L.spg_plan_destroy(plan) == 0
    # options out of range
    o = B.make_options(hash_max_flops=1 << 20)
    assert L.spg_plan_create(ctypes.byref(A), ctypes.byref(Bm), 4, ctypes.byref(o), None,
                             ctypes.byref(plan)) == 1


def test_noalloc_prune_count_refuses_oversize_on_host(lib):
    """More slices than the no-allocation scratch serves: SPG_E_NOMEM before
    any HIP call (the descriptor's arrays are never read)."""
    from paper_2106_14402_amd import binding as B

    L = B.load(LIB)
    dummy = ctypes.c_void_p(0x1000)
    C = B.spg_matrix(4, B.SPG_NOALLOC_MAX_SLICES + 1, 0, B.SPG_CSC, dummy.value, dummy.value, dummy.value)
    nnz = ctypes.c_int64(-1)
    st = L.spg_prune_count_f32_noalloc(ctypes.byref(C), ctypes.c_float(1e-4), None, dummy, ctypes.byref(nnz))
    assert st == 5 and nnz.value == -1
