"""Serving loop: frontier-expansion requests against a resident adjacency.

A request is a sparse frontier F (n x k, 1..64 sources per column) and asks
for F' = A^T F over (OR,AND): column c of F' is the union of the
out-neighbour lists of the sources in column c (multi-source breadth-first
expansion, the linear-algebra formulation of graph traversal the paper builds
on, Sec. 1 and Sec. 4).  The resident CSC arrays of A^T are the CSR arrays
of A, so the product runs as F'^T = F^T A with F^T in CSR.

Continuous batching: worker threads, each with its own stream, take every
admitted request that is waiting when they become free, concatenate their
frontier rows into one left operand and run one product; requests that
arrive meanwhile are admitted as memory frees up and go to the next free
worker, so batches overlap on the device.  Admission is by an HBM budget
against an upper bound of each request's footprint.  The semiring
arithmetic is the library's, identical alone or in a batch.
"""
from __future__ import annotations

import collections
import dataclasses
import threading
import time
from typing import List, Optional

import numpy as np
import torch

from . import binding as B_
from .spgemm import DeviceMatrix, Product

SPG_OK, SPG_E_INVALID, SPG_E_NOMEM, SPG_E_DEVICE = 0, 1, 5, 7
# Statuses of the server itself (not the library's): a request withdrawn by
# cancel() before a worker took it, and one whose deadline passed while it
# waited.
CANCELLED, EXPIRED = -1, -2


@dataclasses.dataclass
class Result:
    rid: int
    status: int
    arrival: float = 0.0
    start: float = 0.0
    done: float = 0.0
    ptr: Optional[np.ndarray] = None   # k+1 offsets (F'^T rows)
    idx: Optional[np.ndarray] = None   # column ids, sorted per row
    flops: int = 0
    batch_rows: int = 0

    @property
    def latency(self) -> float:
        return self.done - self.arrival


class ResidentGraph:
    """The adjacency kept in HBM (pattern-only CSR of out-neighbour lists),
    its host degree array for admission bounds, and panel indexes built once.
    The operand is checked on the device once, at load; the plans that use it
    skip that check (options.b_checked)."""

    def __init__(self, A_host, device="cuda", options=None):
        assert A_host.layout == "csr"
        self.n = A_host.nrows
        self.outdeg = np.diff(A_host.ptr).astype(np.int64)
        self.device = torch.device(device)
        self.A = DeviceMatrix(A_host.nrows, A_host.ncols, "csr",
                              torch.from_numpy(A_host.ptr).to(self.device),
                              torch.from_numpy(A_host.idx).to(self.device), None)
        scratch = torch.zeros(64, dtype=torch.int32, device=self.device)
        flags = B_.spg_matrix_check(self.A.descriptor(), scratch)
        if flags:
            raise ValueError(f"resident operand fails the device check (error bits {flags})")
        self.options = B_.make_options(b_checked=1) if options is None else options
        self.options.b_checked = 1
        self._panels = {}
        self._lock = threading.Lock()

    def panels(self, wlog2: int, stream=None) -> torch.Tensor:
        with self._lock:
            if wlog2 not in self._panels:
                d = self.A.descriptor()
                nb = B_.spg_panel_index_size(d, wlog2)
                t = torch.empty(max(4, nb), dtype=torch.uint8, device=self.device)
                B_.spg_panel_index_build(d, wlog2, t, stream)
                torch.cuda.current_stream(self.device).synchronize() if stream is None else stream.synchronize()
                self._panels[wlog2] = t
            return self._panels[wlog2]

    def workspace_bytes(self, rows: int, entries: int) -> int:
        """Device workspace of the product of a batch of `rows` frontier rows
        holding `entries` sources: the size the library reports for that plan
        (plan creation is host-only and reads only the descriptors)."""
        return plan_workspace_bytes(self.A.descriptor(), self.n, rows, entries, self.options)


def plan_workspace_bytes(Adesc, n: int, rows: int, entries: int, options) -> int:
    """Workspace of F^T (rows x n, `entries` entries) times the resident
    operand, from a plan created for the descriptors alone and destroyed."""
    F = B_.spg_matrix(int(rows), int(n), int(entries), B_.SPG_CSR, Adesc.ptr, Adesc.idx if entries else None,
                      None)
    plan = B_.spg_plan_create(F, Adesc, "or_and_bool", options, 0)
    try:
        return B_.spg_workspace_size(plan)
    finally:
        B_.spg_plan_destroy(plan)


def request_bound_bytes(graph: ResidentGraph, Ft) -> int:
    """Upper bound of a request's device footprint without the workspace: its
    frontier, an output with one entry per product, and offsets.  Admission
    adds the workspace of the whole batch (ResidentGraph.workspace_bytes)."""
    k = Ft.nrows
    flops = int(graph.outdeg[Ft.idx].sum()) if Ft.nnz else 0
    return 12 * Ft.nnz + 8 * (k + 1) + 4 * flops + 8 * (k + 1) + 4096


def check_frontier(graph: ResidentGraph, Ft) -> bool:
    """Host check of a request before admission: shape, ids in range, ids
    strictly ascending per column."""
    if Ft.ncols != graph.n or Ft.layout != "csr":
        return False
    if Ft.ptr[0] != 0 or Ft.ptr[-1] != Ft.nnz or np.any(np.diff(Ft.ptr) < 0):
        return False
    if Ft.nnz == 0:
        return True
    if Ft.idx.min() < 0 or Ft.idx.max() >= graph.n:
        return False
    d = np.diff(Ft.idx.astype(np.int64))
    row_start = np.zeros(Ft.nnz, bool)
    row_start[Ft.ptr[:-1][np.diff(Ft.ptr) > 0]] = True
    return bool(np.all((d > 0) | row_start[1:]))


class FrontierServer:
    def __init__(self, graph: ResidentGraph, hbm_budget: int = 4 << 30, max_batch_rows: int = 8192,
                 max_batch_requests: int = 256, workers: int = 2, options=None):
        self.g = graph
        self.budget = int(hbm_budget)
        self.max_rows = max_batch_rows
        self.max_reqs = max_batch_requests
        self.nworkers = workers
        # plans skip the check of the resident operand (checked at load)
        self.options = B_.make_options(b_checked=1) if options is None else options
        self.options.b_checked = 1
        self._cv = threading.Condition()
        self._pending = collections.deque()   # (arrival, rid, Ft, bound)
        self._deadline = {}                   # rid -> time after which it is not started
        self._in_flight = 0
        self._results: List[Result] = []
        self._stop = False
        self._feeding = False

    # ---- admission ---------------------------------------------------------
    def workspace_bytes(self, rows: int, entries: int) -> int:
        """Workspace of the product of a batch of `rows` frontier rows with
        `entries` sources, as the library sizes it for this server's options."""
        return plan_workspace_bytes(self.g.A.descriptor(), self.g.n, rows, entries, self.options)

    def _take_batch(self):
        """Block until at least one request fits the budget, then take every
        waiting request that fits (FIFO) up to the batch caps.  A batch's
        admitted bytes are its requests' bounds plus the workspace of its
        product."""
        with self._cv:
            while True:
                self._expire_locked(time.perf_counter())
                if self._pending:
                    batch, rows, ents, need = [], 0, 0, 0
                    while self._pending and len(batch) < self.max_reqs:
                        arr, rid, Ft, bound = self._pending[0]
                        if batch and rows + Ft.nrows > self.max_rows:
                            break
                        ws = self.workspace_bytes(rows + Ft.nrows, ents + Ft.nnz)
                        if self._in_flight + need + bound + ws > self.budget:
                            break
                        self._pending.popleft()
                        self._deadline.pop(rid, None)  # taken: it runs to completion
                        batch.append((arr, rid, Ft, bound))
                        rows += Ft.nrows
                        ents += Ft.nnz
                        need += bound
                    if batch:
                        need += self.workspace_bytes(rows, ents)
                        self._in_flight += need
                        return batch, need
                if self._stop and not self._feeding and not self._pending:
                    return None, 0
                self._cv.wait(timeout=0.05)

    def _expire_locked(self, now: float) -> None:
        """Drop the waiting requests whose deadline has passed (caller holds
        the lock); each gets an EXPIRED result."""
        if not self._deadline:
            return
        keep = collections.deque()
        for item in self._pending:
            arr, rid, _, _ = item
            dl = self._deadline.get(rid)
            if dl is not None and now > dl:
                self._results.append(Result(rid, EXPIRED, arr, now, now))
                del self._deadline[rid]
            else:
                keep.append(item)
        self._pending = keep

    def cancel(self, rid: int) -> bool:
        """Withdraw a request that no worker has taken yet; it completes with
        status CANCELLED.  False if it is not waiting (already taken,
        finished or unknown): a product under way is not interrupted."""
        with self._cv:
            for item in self._pending:
                if item[1] == rid:
                    self._pending.remove(item)
                    self._deadline.pop(rid, None)
                    now = time.perf_counter()
                    self._results.append(Result(rid, CANCELLED, item[0], now, now))
                    self._cv.notify_all()
                    return True
        return False

    def _release(self, need):
        with self._cv:
            self._in_flight -= need
            self._cv.notify_all()

    def submit(self, rid: int, Ft, arrival: float, deadline: Optional[float] = None) -> Optional[Result]:
        """Queue a request; returns a Result right away when it is rejected.
        deadline: a time.perf_counter() value after which the request is not
        started any more (it then completes with status EXPIRED)."""
        if not check_frontier(self.g, Ft):
            return Result(rid, SPG_E_INVALID, arrival, arrival, time.perf_counter())
        bound = request_bound_bytes(self.g, Ft)
        if bound + self.workspace_bytes(Ft.nrows, Ft.nnz) > self.budget:
            return Result(rid, SPG_E_NOMEM, arrival, arrival, time.perf_counter())
        with self._cv:
            self._pending.append((arrival, rid, Ft, bound))
            if deadline is not None:
                self._deadline[rid] = deadline
            self._cv.notify_all()
        return None

    # ---- execution ---------------------------------------------------------
    def _execute(self, batch, stream) -> List[Result]:
        start = time.perf_counter()
        ks = [Ft.nrows for _, _, Ft, _ in batch]
        ptrs, idxs, base = [np.zeros(1, np.int64)], [], 0
        for _, _, Ft, _ in batch:
            ptrs.append(Ft.ptr[1:] + base)
            idxs.append(Ft.idx)
            base += Ft.nnz
        ptr_h = np.concatenate(ptrs)
        idx_h = np.concatenate(idxs) if idxs else np.zeros(0, np.int32)
        ktot = int(sum(ks))
        dev = self.g.device
        with torch.cuda.stream(stream):
            F = DeviceMatrix(ktot, self.g.n, "csr", torch.from_numpy(ptr_h).to(dev, non_blocking=False),
                             torch.from_numpy(idx_h.astype(np.int32)).to(dev, non_blocking=False), None)
            prod = Product(F, self.g.A, "or_and_bool", self.options, stream)
            try:
                sw, sp, nw, npn = B_.spg_plan_panels(prod.plan)
                if sp > 1:
                    B_.spg_plan_set_panels(prod.plan, 0, self.g.panels(sw, stream), sw)
                if npn > 1:
                    B_.spg_plan_set_panels(prod.plan, 1, self.g.panels(nw, stream), nw)
                prod.symbolic()
                C = prod.numeric()
                flops = prod.stats()[0]
                cptr = C.ptr.to("cpu")
                cidx = C.idx.to("cpu")
                stream.synchronize()
            finally:
                prod.close()
        done = time.perf_counter()
        cptr = cptr.numpy()
        cidx = cidx.numpy()
        out, row = [], 0
        for (arr, rid, Ft, _), k in zip(batch, ks):
            lo, hi = int(cptr[row]), int(cptr[row + k])
            rptr = cptr[row:row + k + 1] - lo
            f = int(self.g.outdeg[Ft.idx].sum()) if Ft.nnz else 0
            out.append(Result(rid, SPG_OK, arr, start, done, rptr, cidx[lo:hi].copy(), f, ktot))
            row += k
        return out

    def _worker(self):
        self._worker_loop(torch.cuda.Stream(self.g.device))

    def _worker_loop(self, stream):
        while True:
            batch, need = self._take_batch()
            if batch is None:
                return
            try:
                res = self._execute(batch, stream)
            except B_.SpgError as e:
                now = time.perf_counter()
                res = [Result(rid, e.status, arr, now, now) for arr, rid, _, _ in batch]
            except Exception:  # noqa: BLE001 - a failed batch must not drop its requests
                now = time.perf_counter()
                res = [Result(rid, SPG_E_DEVICE, arr, now, now) for arr, rid, _, _ in batch]
            finally:
                self._release(need)
            with self._cv:
                self._results.extend(res)

    def serve(self, requests, rate_scale: float = 1.0, timeout_s: Optional[float] = None) -> List[Result]:
        """Replay ``requests`` (each with .rid, .arrival seconds, .Ft) in real
        time and return every result (completed, rejected or, with
        timeout_s, expired after waiting that long)."""
        self._results = []
        self._stop = False
        self._feeding = True
        threads = [threading.Thread(target=self._worker, daemon=True) for _ in range(self.nworkers)]
        for t in threads:
            t.start()
        t0 = time.perf_counter()
        rejected = []
        for r in requests:
            target = t0 + r.arrival * rate_scale
            delay = target - time.perf_counter()
            if delay > 0:
                time.sleep(delay)
            rej = self.submit(r.rid, r.Ft, target, None if timeout_s is None else target + timeout_s)
            if rej is not None:
                rejected.append(rej)
        with self._cv:
            self._feeding = False
            self._stop = True
            self._cv.notify_all()
        for t in threads:
            t.join()
        return sorted(self._results + rejected, key=lambda x: x.rid)


def expand_alone(graph: ResidentGraph, Ft, options=None):
    """One request through its own product (the reference for 'alone')."""
    dev = graph.device
    F = DeviceMatrix(Ft.nrows, graph.n, "csr", torch.from_numpy(Ft.ptr).to(dev),
                     torch.from_numpy(Ft.idx.astype(np.int32)).to(dev), None)
    prod = Product(F, graph.A, "or_and_bool", options or graph.options)
    try:
        prod.symbolic()
        C = prod.numeric()
        torch.cuda.synchronize()
        return C.ptr.cpu().numpy(), C.idx.cpu().numpy()
    finally:
        prod.close()


def latency_summary(results: List[Result], t_first: Optional[float] = None) -> dict:
    ok = [r for r in results if r.status == SPG_OK]
    if not ok:
        return {"completed": 0}
    lat = np.array([r.latency for r in ok]) * 1e3
    t0 = min(r.arrival for r in ok) if t_first is None else t_first
    span = max(r.done for r in ok) - t0
    flops = sum(r.flops for r in ok)
    return {
        "completed": len(ok),
        "rejected": len(results) - len(ok),
        "p50_ms": float(np.percentile(lat, 50)),
        "p99_ms": float(np.percentile(lat, 99)),
        "mean_ms": float(lat.mean()),
        "req_per_s": len(ok) / span,
        "gflops": 2.0 * flops / span / 1e9,
        "mean_batch_rows": float(np.mean([r.batch_rows for r in ok])),
    }
