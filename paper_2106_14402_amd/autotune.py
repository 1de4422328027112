"""Autotuner for batched products.

The batched plan's launch shape is set by a handful of knobs: the symbolic
bin threshold between LDS hash tables and bitmap rows (hash_max_flops), the
largest numeric hash table (hash_max_nnz, which sets the table sizes used),
the segment length above which B rows are split across waves (short_seg),
the workgroup size of the dense kernels (dense_threads) and the LDS given to
a dense value panel (lds_budget, which sets the panel width).  The best
values depend on the mix of products and on the device, so they are found
by timing: coordinate descent from the library defaults, one knob at a
time, each candidate timed on the batch itself (symbolic + numeric, median
of a few runs).  Only launch shapes change; the arithmetic of every
semiring is the same under every candidate.

Winners are kept in a JSON cache keyed by the device name and a coarse
signature of the batch (semiring mix, log2 histograms of row counts and of
nonzeros), so a later batch of the same shape reuses them without timing.
"""
from __future__ import annotations

import json
import math
import os
import time
from typing import Dict, List, Optional, Sequence

import numpy as np
import torch

from . import binding as B_

# Library defaults of the batched plan, and the candidates tried per knob.
BATCH_DEFAULTS: Dict[str, int] = {"hash_max_flops": 8192, "hash_max_nnz": 2048, "short_seg": 16,
                                  "dense_threads": 512, "lds_budget": 65536, "esc_ratio_x16": 20}
CANDIDATES: Dict[str, List[int]] = {
    "hash_max_nnz": [512, 1024, 2048, 4096],
    "hash_max_flops": [2048, 4096, 8192, 16384],
    "short_seg": [8, 16, 32, 64],
    "dense_threads": [256, 512, 1024],
    "lds_budget": [32768, 65536, 131072],
    "esc_ratio_x16": [16, 20, 32],
}
ORDER = ["hash_max_nnz", "hash_max_flops", "short_seg", "dense_threads", "lds_budget", "esc_ratio_x16"]

DEFAULT_CACHE = os.path.join(os.path.expanduser("~"), ".cache", "spg_autotune.json")


def _hist_log2(values) -> List[int]:
    h = [0] * 33
    for v in values:
        h[0 if v <= 0 else min(32, int(math.log2(v)) + 1)] += 1
    while h and h[-1] == 0:
        h.pop()
    return h


def signature(As, Bs, semirings: Sequence[str], device_name: str) -> str:
    """Device, semiring mix, and log2 histograms of the operands' row counts
    and nonzeros (matrices may be host SparseMatrix or DeviceMatrix)."""
    mix: Dict[str, int] = {}
    for s in semirings:
        mix[s] = mix.get(s, 0) + 1
    rows = [a.nrows for a in As]
    nnz = [int(a.nnz) + int(b.nnz) for a, b in zip(As, Bs)]
    key = {"device": device_name, "mix": sorted(mix.items()), "rows": _hist_log2(rows),
           "nnz": _hist_log2(nnz), "n": len(As)}
    return json.dumps(key, sort_keys=True)


def load_cache(path: str) -> dict:
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def store_cache(path: str, cache: dict) -> None:
    d = os.path.dirname(path)
    if d:
        os.makedirs(d, exist_ok=True)
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(cache, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def make_options(knobs: Dict[str, int]) -> B_.spg_options:
    return B_.make_options(**knobs)


def time_batch(As, Bs, semirings, knobs: Dict[str, int], reps: int = 3) -> Optional[float]:
    """Median ms of symbolic + numeric for the batch under these knobs, or
    None when the plan rejects them."""
    from .batch import BatchProduct
    try:
        bp = BatchProduct(As, Bs, semirings, make_options(knobs))
    except B_.SpgError:
        return None
    try:
        bp.symbolic()
        bp.allocate()
        bp.numeric()  # warm-up
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
        for e0, e1 in ev:
            e0.record(bp.stream)
            bp.symbolic()
            bp.numeric()
            e1.record(bp.stream)
        torch.cuda.synchronize()
        return float(np.median([e0.elapsed_time(e1) for e0, e1 in ev]))
    except B_.SpgError:
        return None
    finally:
        bp.close()


def tune_batch(As, Bs, semirings, cache_path: Optional[str] = DEFAULT_CACHE, reps: int = 3,
               sweeps: int = 1, force: bool = False, log=None) -> Dict[str, object]:
    """Knob values for this batch: from the cache when its signature is
    there (unless force), else by coordinate descent.  Returns a record with
    the knobs, the tuned and default times, and whether it came from the
    cache."""
    dev = torch.cuda.get_device_name(As[0].ptr.device) if As else "none"
    key = signature(As, Bs, semirings, dev)
    cache = load_cache(cache_path) if cache_path else {}
    if not force and key in cache:
        rec = dict(cache[key])
        rec["from_cache"] = True
        return rec
    t0 = time.time()
    best = dict(BATCH_DEFAULTS)
    default_ms = time_batch(As, Bs, semirings, best, reps)
    best_ms = default_ms
    tried = {json.dumps(best, sort_keys=True): default_ms}
    for _ in range(sweeps):
        for knob in ORDER:
            for v in CANDIDATES[knob]:
                cand = dict(best)
                cand[knob] = v
                k = json.dumps(cand, sort_keys=True)
                if k not in tried:
                    tried[k] = time_batch(As, Bs, semirings, cand, reps)
                    if log:
                        log(f"[autotune] {knob}={v}: {tried[k]}")
                ms = tried[k]
                if ms is not None and (best_ms is None or ms < best_ms):
                    best, best_ms = cand, ms
    rec = {"knobs": best, "ms": best_ms, "default_ms": default_ms, "evaluated": len(tried),
           "tune_s": round(time.time() - t0, 2)}
    if cache_path:
        cache = load_cache(cache_path)
        cache[key] = rec
        store_cache(cache_path, cache)
    rec = dict(rec)
    rec["from_cache"] = False
    return rec
