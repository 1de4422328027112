"""Seeded synthetic sparse-matrix generators.

This module is shared by the CPU oracle tests and the GPU path.  It holds no
part of the semiring product itself: it only draws sparsity patterns and
values, and packs them into compressed sparse row / column arrays.

Workloads (stand-ins for the paper's matrices, none of which are available):

* Erdos-Renyi: a fixed number of distinct uniformly drawn columns per row.
* R-MAT (recursive-matrix) graphs with Graph500-style quadrant probabilities,
  the skewed-degree family the paper uses for its graph experiments (Sec. 4,
  SpMSpV study; random vertex relabelling for balance, Sec. 3.1).
* A column-stochastic Markov-clustering matrix with log-normal column
  degrees, the operand of HipMCL's expansion step (Sec. 7, HipMCL study).
* A mix of many uneven products (one GPU's share of a 3D SUMMA stage, Sec. 3).
* A Poisson stream of sparse frontier matrices for a resident adjacency
  matrix (multi-source breadth-first expansion).

Every generator takes a ``numpy.random.Generator`` (or a seed) so results are
reproducible bit for bit.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Tuple

import numpy as np

SEED_BASE = 2106_14402


def rng_for(config: int, sub: int = 0) -> np.random.Generator:
    """Generator for workload ``config`` (0-based) and sub-item ``sub``."""
    return np.random.default_rng(SEED_BASE + config + 1000 * sub)


def _rng(r) -> np.random.Generator:
    return r if isinstance(r, np.random.Generator) else np.random.default_rng(r)


@dataclasses.dataclass
class SparseMatrix:
    """Compressed sparse matrix with int64 offsets and int32 indices.

    ``layout == "csr"``: ``ptr`` has ``nrows + 1`` entries and ``idx`` holds
    column indices.  ``layout == "csc"``: ``ptr`` has ``ncols + 1`` entries and
    ``idx`` holds row indices.  ``val`` is ``None`` for a pattern-only boolean
    matrix (every stored entry is true).
    """

    nrows: int
    ncols: int
    layout: str
    ptr: np.ndarray
    idx: np.ndarray
    val: Optional[np.ndarray]

    @property
    def nnz(self) -> int:
        return int(self.idx.shape[0])

    @property
    def nmajor(self) -> int:
        return self.nrows if self.layout == "csr" else self.ncols

    @property
    def nminor(self) -> int:
        return self.ncols if self.layout == "csr" else self.nrows

    def degrees(self) -> np.ndarray:
        return np.diff(self.ptr)

    def with_values(self, val: Optional[np.ndarray]) -> "SparseMatrix":
        return dataclasses.replace(self, val=val)

    def transpose_view(self) -> "SparseMatrix":
        """The same arrays read as the transpose in the other layout."""
        lay = "csc" if self.layout == "csr" else "csr"
        return SparseMatrix(self.ncols, self.nrows, lay, self.ptr, self.idx, self.val)


def from_pairs(nrows: int, ncols: int, major: np.ndarray, minor: np.ndarray,
               val: Optional[np.ndarray], layout: str = "csr",
               presorted: bool = False) -> SparseMatrix:
    """Pack (major, minor) pairs without duplicates into a compressed matrix,
    minor indices ascending within each major slice."""
    nmajor = nrows if layout == "csr" else ncols
    nminor = ncols if layout == "csr" else nrows
    major = np.asarray(major, dtype=np.int64)
    minor = np.asarray(minor, dtype=np.int64)
    if not presorted and major.size:
        order = np.lexsort((minor, major))
        major = major[order]
        minor = minor[order]
        if val is not None:
            val = np.asarray(val)[order]
    counts = np.bincount(major, minlength=nmajor) if major.size else np.zeros(nmajor, np.int64)
    ptr = np.zeros(nmajor + 1, dtype=np.int64)
    np.cumsum(counts, out=ptr[1:])
    idx = minor.astype(np.int32)
    assert nminor <= 2**31 - 1
    return SparseMatrix(nrows, ncols, layout, ptr, idx,
                        None if val is None else np.ascontiguousarray(val))


def distinct_minor(nmajor: int, nminor: int, degs: np.ndarray, rng) -> Tuple[np.ndarray, np.ndarray]:
    """Per major slice ``r``, draw ``degs[r]`` distinct minor indices uniformly
    without replacement.  Returns (major, minor) sorted by (major, minor)."""
    rng = _rng(rng)
    degs = np.minimum(np.asarray(degs, dtype=np.int64), nminor)
    major = np.repeat(np.arange(nmajor, dtype=np.int64), degs)
    minor = rng.integers(0, nminor, size=major.size, dtype=np.int64)
    while True:
        key = major * nminor + minor
        order = np.argsort(key, kind="stable")
        key = key[order]
        minor = minor[order]
        dup = np.zeros(key.size, dtype=bool)
        if key.size > 1:
            dup[1:] = key[1:] == key[:-1]
        ndup = int(dup.sum())
        if ndup == 0:
            return major, minor
        minor[dup] = rng.integers(0, nminor, size=ndup, dtype=np.int64)


# --------------------------------------------------------------------------
# Erdos-Renyi
# --------------------------------------------------------------------------
def erdos_renyi(n: int, d: int, rng, values: str = "f64", ncols: Optional[int] = None) -> SparseMatrix:
    """``n`` rows with exactly ``d`` distinct columns each, drawn uniformly
    without replacement (self loops allowed).  ``values``: ``"f64"`` U[0,1),
    ``"i32"`` integers U[1,255], ``"f32"`` U[0,1), ``"bool"`` ones, ``None``
    pattern only."""
    rng = _rng(rng)
    ncols = n if ncols is None else ncols
    major, minor = distinct_minor(n, ncols, np.full(n, d, dtype=np.int64), rng)
    val = draw_values(values, major.size, rng)
    return from_pairs(n, ncols, major, minor, val, "csr", presorted=True)


def draw_values(kind: Optional[str], count: int, rng) -> Optional[np.ndarray]:
    rng = _rng(rng)
    if kind is None:
        return None
    if kind == "f64":
        return rng.random(count, dtype=np.float64)
    if kind == "f32":
        return rng.random(count, dtype=np.float32)
    if kind == "i32":
        return rng.integers(1, 256, size=count, dtype=np.int32)
    if kind == "bool":
        return np.ones(count, dtype=np.uint8)
    raise ValueError(kind)


# --------------------------------------------------------------------------
# R-MAT
# --------------------------------------------------------------------------
def rmat_draw(scale: int, nedges: int, a: float, b: float, c: float, rng) -> Tuple[np.ndarray, np.ndarray]:
    """Draw ``nedges`` R-MAT edges over ``2**scale`` vertices: at every level
    one of four quadrants is taken with probabilities a, b, c, 1-a-b-c (no
    per-level noise).  Returns (src, dst) as int64."""
    rng = _rng(rng)
    src = np.zeros(nedges, dtype=np.int64)
    dst = np.zeros(nedges, dtype=np.int64)
    ab, abc = a + b, a + b + c
    for lev in range(scale):
        u = rng.random(nedges, dtype=np.float64)
        hi = u >= ab
        right = (u >= a) & ~hi | (u >= abc)
        bit = np.int64(1) << np.int64(lev)
        src |= hi.astype(np.int64) * bit
        dst |= right.astype(np.int64) * bit
    return src, dst


def rmat_graph(scale: int, edge_factor: int, rng, a: float = 0.57, b: float = 0.19, c: float = 0.19,
               symmetric: bool = True, weights: Optional[str] = None, permute: bool = True,
               n: Optional[int] = None, layout: str = "csr") -> SparseMatrix:
    """R-MAT adjacency matrix.

    ``n`` (default ``2**scale``) lets the vertex count be a non-power of two:
    edges are drawn at scale ``ceil(log2 n)`` and any edge with an endpoint
    ``>= n`` is redrawn until ``n * edge_factor`` draws are kept.  Self loops and
    duplicates are removed; ``symmetric`` adds the reverse of every edge
    (weights are then shared by both directions).  Vertex ids are relabelled
    by a seeded random permutation when ``permute``.

    ``weights``: ``None`` (pattern only), ``"i32"`` U[1,255], ``"f64"`` U[0,1),
    ``"bool"`` all ones.
    """
    rng = _rng(rng)
    if n is None:
        n = 1 << scale
    else:
        scale = max(1, int(math.ceil(math.log2(n))))
    want = n * edge_factor
    srcs, dsts, got = [], [], 0
    while got < want:
        s, d = rmat_draw(scale, want - got, a, b, c, rng)
        keep = (s < n) & (d < n)
        srcs.append(s[keep])
        dsts.append(d[keep])
        got += int(keep.sum())
    src = np.concatenate(srcs)
    dst = np.concatenate(dsts)
    if permute:
        perm = rng.permutation(n).astype(np.int64)
        src = perm[src]
        dst = perm[dst]
    keep = src != dst
    src, dst = src[keep], dst[keep]
    if symmetric:
        lo = np.minimum(src, dst)
        hi = np.maximum(src, dst)
        key = np.unique(lo * n + hi)
        lo, hi = key // n, key % n
        w = draw_values(weights, key.size, rng)
        major = np.concatenate([lo, hi])
        minor = np.concatenate([hi, lo])
        val = None if w is None else np.concatenate([w, w])
        key = major * n + minor
        order = np.argsort(key, kind="stable")
        major, minor = major[order], minor[order]
        val = None if val is None else val[order]
    else:
        key = np.unique(src * n + dst)
        major, minor = key // n, key % n
        val = draw_values(weights, key.size, rng)
    if layout == "csc":
        # A directed graph stored by columns: same (src, dst) pairs, minor = src.
        return from_pairs(n, n, minor, major, val, "csc")
    return from_pairs(n, n, major, minor, val, "csr", presorted=True)


# --------------------------------------------------------------------------
# Markov-clustering (column-stochastic) matrix
# --------------------------------------------------------------------------
def mcl_matrix(n: int, mean_deg: float, sigma: float, rng) -> SparseMatrix:
    """Column-stochastic CSC float32 matrix.

    Column degrees are ``clamp(round(LogNormal(ln(mean_deg) - sigma^2/2, sigma)), 1, n)``
    (so the mean is ``mean_deg``); row ids per column are uniform without
    replacement; values are LogNormal(0, 1), normalised per column in float64
    and rounded to float32."""
    rng = _rng(rng)
    mu = math.log(mean_deg) - 0.5 * sigma * sigma
    degs = np.clip(np.rint(rng.lognormal(mu, sigma, size=n)), 1, n).astype(np.int64)
    col, row = distinct_minor(n, n, degs, rng)
    raw = rng.lognormal(0.0, 1.0, size=col.size)
    colsum = np.bincount(col, weights=raw, minlength=n)
    val = (raw / colsum[col]).astype(np.float32)
    return from_pairs(n, n, col, row, val, "csc", presorted=True)


# --------------------------------------------------------------------------
# Batched mix of uneven products
# --------------------------------------------------------------------------
@dataclasses.dataclass
class BatchItem:
    index: int
    graph: str          # "er" or "rmat"
    semiring: str       # "plus_times_f64" or "min_plus_i32"
    n: int
    degree: int
    A: SparseMatrix


def batch_mix(nprod: int = 512, n_lo: int = 1024, n_hi: int = 65536, d_lo: int = 4, d_hi: int = 32,
              config: int = 3) -> List[BatchItem]:
    """``nprod`` squaring products of uneven size.  Item ``b``: Erdos-Renyi when
    ``b`` is even, directed R-MAT (a=.57, b=.19, c=.19) when odd; semiring
    (+,x) float64 when ``b // 2`` is even, (min,+) int32 otherwise; ``n``
    log-uniform in [n_lo, n_hi]; degree uniform integer in [d_lo, d_hi]."""
    items = []
    for bi in range(nprod):
        rng = rng_for(config, bi)
        n = int(round(math.exp(rng.uniform(math.log(n_lo), math.log(n_hi)))))
        d = int(rng.integers(d_lo, d_hi + 1))
        semiring = "plus_times_f64" if (bi // 2) % 2 == 0 else "min_plus_i32"
        vals = "f64" if semiring == "plus_times_f64" else "i32"
        if bi % 2 == 0:
            A = erdos_renyi(n, d, rng, values=vals)
            g = "er"
        else:
            A = rmat_graph(0, d, rng, symmetric=False, weights=vals, n=n)
            g = "rmat"
        items.append(BatchItem(bi, g, semiring, n, d, A))
    return items


# --------------------------------------------------------------------------
# Served request stream
# --------------------------------------------------------------------------
@dataclasses.dataclass
class Request:
    rid: int
    arrival: float       # seconds from stream start
    k: int               # number of frontier columns
    Ft: SparseMatrix     # the frontier F^T in CSR: row c = sources of column c


def frontier(n: int, k: int, rng, max_sources: int = 64) -> SparseMatrix:
    """Frontier F (n x k) returned as F^T in CSR (k x n): each of the ``k``
    columns holds 1..max_sources distinct uniformly drawn source vertices."""
    rng = _rng(rng)
    cnt = rng.integers(1, max_sources + 1, size=k, dtype=np.int64)
    major, minor = distinct_minor(k, n, cnt, rng)
    return from_pairs(k, n, major, minor, None, "csr", presorted=True)


def request_stream(n: int, count: int, rate: float, rng, k_max: int = 1024,
                   max_sources: int = 64) -> List[Request]:
    """``count`` requests with exponential inter-arrival times of mean
    ``1/rate`` seconds and widths ``k = round(exp(U(0, ln k_max)))``."""
    rng = _rng(rng)
    gaps = rng.exponential(1.0 / rate, size=count)
    t = np.cumsum(gaps)
    out = []
    for r in range(count):
        k = int(round(math.exp(rng.uniform(0.0, math.log(k_max)))))
        out.append(Request(r, float(t[r]), k, frontier(n, k, rng, max_sources)))
    return out


# --------------------------------------------------------------------------
# The five named workloads
# --------------------------------------------------------------------------
def config_er(n: int = 4096, d: int = 8) -> SparseMatrix:
    """Erdos-Renyi n=4096, 8 distinct columns per row, float64 U[0,1), CSR."""
    return erdos_renyi(n, d, rng_for(0), values="f64")


def config_rmat(scale: int = 20, edge_factor: int = 16) -> SparseMatrix:
    """Symmetrised R-MAT (a=.57,b=.19,c=.19,d=.05) with int32 weights
    U[1,255] shared by both directions of an edge; the boolean workload uses
    the same pattern with ``val=None``."""
    return rmat_graph(scale, edge_factor, rng_for(1), symmetric=True, weights="i32")


def config_mcl(n: int = 1 << 20, mean_deg: float = 48.0, sigma: float = 1.0) -> SparseMatrix:
    return mcl_matrix(n, mean_deg, sigma, rng_for(2))


def config_served_graph(scale: int = 22, edge_factor: int = 16) -> SparseMatrix:
    """Directed R-MAT adjacency, pattern only, CSR (out-neighbour lists)."""
    return rmat_graph(scale, edge_factor, rng_for(4), symmetric=False, weights=None)
