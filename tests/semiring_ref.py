"""Dense brute-force semiring products for tiny inputs (test helper).

Independent of the oracle: it expands the definition of the semiring product
into a dense (m, n, k) tensor of all products A(i,k) (x) B(k,j), masks it by
the stored pattern of both operands, and folds it over k with (+).  This is
the paper's problem statement C = AB over a semiring (Sec. 3.1) with nothing
else in between.
"""
import numpy as np

INT32_MAX = np.iinfo(np.int32).max
INT32_MIN = np.iinfo(np.int32).min


def dense(M):
    """(values, presence) dense arrays of a spgen.SparseMatrix; missing values
    are reported as ones (pattern-only boolean)."""
    pres = np.zeros((M.nrows, M.ncols), dtype=bool)
    vals = np.zeros((M.nrows, M.ncols), dtype=np.float64 if M.val is None else M.val.dtype)
    for s in range(M.nmajor):
        lo, hi = int(M.ptr[s]), int(M.ptr[s + 1])
        minor = M.idx[lo:hi]
        v = np.ones(hi - lo) if M.val is None else M.val[lo:hi]
        if M.layout == "csr":
            pres[s, minor] = True
            vals[s, minor] = v
        else:
            pres[minor, s] = True
            vals[minor, s] = v
    return vals, pres


def _total_order_key(x):
    """Map floats to int keys whose order is the total order with -0 < +0."""
    x = np.asarray(x)
    if x.dtype == np.float32:
        b = x.view(np.int32).astype(np.int64)
        return np.where(b < 0, -(b & 0x7FFFFFFF) - 1, b)
    b = x.view(np.int64)
    big = np.int64(0x7FFFFFFFFFFFFFFF)
    return np.where(b < 0, -(b & big) - 1, b)


def brute_force(A, B, semiring):
    """Return (presence[m,k], values[m,k]) of C = A (x).(+) B."""
    Av, Ap = dense(A)
    Bv, Bp = dense(B)
    mask = Ap[:, :, None] & Bp[None, :, :]          # (m, n, k)
    pres = mask.any(axis=1)
    m, n = Ap.shape
    k = Bp.shape[1]
    out = np.zeros((m, k), dtype=object)
    if semiring in ("plus_times_f64", "plus_times_f32"):
        a = Av.astype(np.float64)
        b = Bv.astype(np.float64)
        prod = a[:, :, None] * b[None, :, :]
        vals = np.zeros((m, k), np.float64)
        for kk in range(n):                            # left fold over k ascending
            vals = np.where(mask[:, kk, :], vals + prod[:, kk, :], vals)
        return pres, vals
    if semiring == "min_plus_i32":
        s = Av.astype(np.int64)[:, :, None] + Bv.astype(np.int64)[None, :, :]
        s = np.clip(s, INT32_MIN, INT32_MAX)
        s = np.where(mask, s, np.int64(INT32_MAX) + 1)
        vals = s.min(axis=1)
        return pres, np.where(pres, vals, 0).astype(np.int32)
    if semiring in ("min_plus_f32", "max_times_f64", "max_times_f32"):
        if semiring == "min_plus_f32":
            prod = Av.astype(np.float32)[:, :, None] + Bv.astype(np.float32)[None, :, :]
        elif semiring == "max_times_f32":
            prod = Av.astype(np.float32)[:, :, None] * Bv.astype(np.float32)[None, :, :]
        else:
            prod = Av.astype(np.float64)[:, :, None] * Bv.astype(np.float64)[None, :, :]
        key = _total_order_key(prod)
        if semiring == "min_plus_f32":
            key = np.where(mask, key, np.iinfo(np.int64).max)
            pos = key.argmin(axis=1)
        else:
            key = np.where(mask, key, np.iinfo(np.int64).min)
            pos = key.argmax(axis=1)
        vals = np.take_along_axis(prod, pos[:, None, :], axis=1)[:, 0, :]
        return pres, np.where(pres, vals, 0).astype(prod.dtype)
    if semiring == "or_and_bool":
        a = Av != 0
        b = Bv != 0
        prod = a[:, :, None] & b[None, :, :]
        vals = (prod & mask).any(axis=1)
        return pres, vals.astype(np.uint8)
    raise ValueError(semiring)


def to_dense_result(ptr, idx, val, nmajor, nminor, layout, dtype):
    """Scatter a packed (ptr, idx, val) result into dense presence/value arrays
    in (row, column) orientation."""
    pres = np.zeros((nmajor, nminor), bool)
    vals = np.zeros((nmajor, nminor), dtype)
    for s in range(nmajor):
        lo, hi = int(ptr[s]), int(ptr[s + 1])
        assert np.all(np.diff(idx[lo:hi]) > 0), "slice not strictly ascending"
        pres[s, idx[lo:hi]] = True
        vals[s, idx[lo:hi]] = val[lo:hi]
    if layout == "csc":
        return pres.T, vals.T
    return pres, vals
