"""Planted mistakes in a copy of the oracle must fail the pins (CPU only).

Each mutant is the oracle source with one plausible slip (a dropped term, a
wrong sign, a swapped operand, a wrong index, a wrong reduction, a missing
clamp, a wrong tie rule); it is compiled to a temporary library and run
through the same checks that pin the real oracle.  A mutant that passes them
would mean the pins cannot tell that mistake apart from the definition.
"""
import os
import subprocess

import numpy as np
import pytest

import oracle
import spgen
from tests.semiring_ref import brute_force, to_dense_result
from tests.test_oracle_pins import ALL, VALKIND, random_sparse

MUTANTS = {
    "dropped_term_rows": ("for (int64_t q = Bp[k]; q < Bp[k + 1]; ++q)",
                          "for (int64_t q = Bp[k]; q + 1 < Bp[k + 1]; ++q)"),
    "dropped_term_cols": ("for (int64_t p = Ap[k]; p < Ap[k + 1]; ++p)",
                          "for (int64_t p = Ap[k] + 1; p < Ap[k + 1]; ++p)"),
    "wrong_sign": ("static T add(T x, T y) { return x + y; }",
                   "static T add(T x, T y) { return x - y; }"),
    "swapped_operand": ("accumulate(Ai[p], S::mul(value_at<S>(Av, p), b));",
                        "accumulate(Ai[p], S::mul(value_at<S>(Bv, p), b));"),
    "wrong_index": ("accumulate(Bi[q], S::mul(a, value_at<S>(Bv, q)));",
                    "accumulate(Bi[q], S::mul(a, value_at<S>(Bv, p)));"),
    "max_for_min": ("static T add(T x, T y) { return y < x ? y : x; }",
                    "static T add(T x, T y) { return y > x ? y : x; }"),
    "no_saturation": ("if (s > INT32_MAX) s = INT32_MAX;", ""),
    "signed_zero_tie": ("return std::signbit(x) && !std::signbit(y);", "return false;"),
    "first_product_doubled": ("acc.emplace(key, prod);", "acc.emplace(key, S::add(prod, prod));"),
}


def _pins_pass(L) -> bool:
    rng = np.random.default_rng(21)
    try:
        for sr in ALL:
            for layout in ("csr", "csc"):
                A = random_sparse(12, 15, 0.35, rng, VALKIND[sr], layout, signed=True)
                B = random_sparse(15, 10, 0.35, rng, VALKIND[sr], layout, signed=True)
                ptr, idx, val = oracle.spgemm(A, B, sr, _lib=L)
                nmaj, nmin = (12, 10) if layout == "csr" else (10, 12)
                pres, vals = to_dense_result(ptr, idx, val, nmaj, nmin, layout, val.dtype)
                bp, bv = brute_force(A, B, sr)
                if not np.array_equal(pres, bp):
                    return False
                if sr.startswith("plus_times"):
                    _, absv = brute_force(A.with_values(np.abs(A.val)), B.with_values(np.abs(B.val)),
                                          "plus_times_f64")
                    if not np.all(np.abs(vals - bv) <= 1e-13 * absv):
                        return False
                elif not np.array_equal(vals[bp].view(np.uint8), bv[bp].astype(vals.dtype).view(np.uint8)):
                    return False
        # saturation and signed-zero pins
        big = np.iinfo(np.int32).max
        A = spgen.from_pairs(1, 1, np.array([0]), np.array([0]), np.array([big - 5], np.int32))
        B = spgen.from_pairs(1, 1, np.array([0]), np.array([0]), np.array([100], np.int32))
        if oracle.spgemm(A, B, "min_plus_i32", _lib=L)[2][0] != big:
            return False
        A = spgen.from_pairs(1, 2, np.array([0, 0]), np.array([0, 1]), np.array([0.0, -0.0], np.float32))
        B = spgen.from_pairs(2, 1, np.array([0, 1]), np.array([0, 0]), np.array([0.0, -0.0], np.float32))
        if not np.signbit(oracle.spgemm(A, B, "min_plus_f32", _lib=L)[2][0]):
            return False
    except (AssertionError, ValueError, IndexError):
        return False
    return True


def test_real_oracle_passes():
    assert _pins_pass(oracle.lib())


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(name, tmp_path):
    src = open(oracle.SRC).read()
    old, new = MUTANTS[name]
    assert src.count(old) >= 1, f"mutation site for {name} not found"
    mutated = src.replace(old, new, 1)
    cpp = os.path.join(tmp_path, "mutant.cpp")
    so = os.path.join(tmp_path, f"libmutant_{name}.so")
    with open(cpp, "w") as f:
        f.write(mutated)
    subprocess.check_call(["g++", "-O1", "-std=c++17", "-fopenmp", "-ffp-contract=off", "-fPIC",
                           "-shared", cpp, "-o", so])
    assert not _pins_pass(oracle.load(so)), f"pins did not catch mutant {name}"
