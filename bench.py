"""Benchmark of the semiring sparse product on one MI355X.

One step is one pass of the whole product pipeline (flop count and binning,
symbolic phase, offsets scan, numeric phase with in-row ordering) over the
R-MAT scale-20 workload: n = 2^20, edge factor 16, a=.57 b=.19 c=.19 d=.05,
symmetrised, no self loops or duplicates, seeded vertex relabelling.  The
step squares it twice: over (OR,AND) on the pattern alone and over (min,+)
with int32 weights U[1,255].  Inputs are resident in HBM before timing
starts; output buffers are allocated once, outside the timed region.

Prints one JSON line: throughput in GFLOP/s (2 x products / time), with a
roofline entry for the dominant kernel (its algorithmic HBM bytes over its
average duration measured with HIP events on the stream it runs on) and the
oracle timed on the host cores over a bounded row sample.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "SpGEMM GFLOP/s (2·flops) + HBM GB/s vs peak; batched speedup; served p50/p99 ms"


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--scale", type=int, default=20, help="R-MAT scale (20 is the named workload)")
    ap.add_argument("--cpu-seconds", type=float, default=15.0,
                    help="target host time of the oracle sample (0 disables)")
    ap.add_argument("--semirings", default="or_and_bool,min_plus_i32")
    ap.add_argument("--workload", default="rmat",
                    choices=["rmat", "er", "mcl", "batched", "served", "merge", "outbatch", "calib", "counters"],
                    help="rmat (default) is the named benchmark workload; the others are the "
                         "remaining configurations, printed in the same JSON form")
    ap.add_argument("--batches", type=int, default=4, help="outbatch: output budget = nnz(C) / batches")
    ap.add_argument("--nprod", type=int, default=512, help="batched: number of products")
    ap.add_argument("--requests", type=int, default=2000, help="served: requests per arrival rate")
    ap.add_argument("--batch-knobs", default="",
                    help="batched: knob values k=v,... instead of the autotuner's")
    ap.add_argument("--autotune-cache", default=None,
                    help="batched: autotuner cache file (default gpurun_out/autotune.json under the repo)")
    ap.add_argument("--opt", action="append", default=[],
                    help="extra option for both products, key=value (e.g. short_seg=16)")
    ap.add_argument("--bitmap-mib", type=int, default=28672,
                    help="workspace for symbolic bitmaps kept for the pattern-only numeric phase")
    ap.add_argument("--bitmap-mib-valued", type=int, default=28672,
                    help="workspace for symbolic bitmaps kept for the rank passes of the (min,+) product")
    ap.add_argument("--select", type=int, default=1100, help="mcl: entries kept per column by the selection")
    ap.add_argument("--counter-dirs", default="",
                    help="counters: read-pass and write-pass rocprofv3 output directories of the workload, "
                         "then those of the calibration run (comma separated)")
    ap.add_argument("--counter-out", default=None, help="counters: summary JSON to write")
    ap.add_argument("--counter-workload", default="rmat20", help="counters: workload name of the summary")
    ap.add_argument("--counter-command", default="", help="counters: the profiled command, for the record")
    return ap.parse_args()


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def kernel_sources_digest():
    """sha256 over the HIP sources of the library: counter figures taken on
    other sources no longer describe the kernels."""
    import hashlib
    h = hashlib.sha256()
    d = os.path.join(ROOT, "paper_2106_14402_amd", "csrc")
    for name in sorted(os.listdir(d)):
        if name.endswith((".hip", ".h")):
            with open(os.path.join(d, name), "rb") as f:
                h.update(name.encode() + b"\0" + f.read())
    return h.hexdigest()


def measured_traffic(kernel, workload, launches=1):
    """HBM bytes of one phase of ``kernel`` from the committed rocprofv3
    counter summary (request counts by size, see run_counters): its mean
    bytes per dispatch times the phase's launches (one per accumulator class;
    a name with several semirings, ``k<a+b>``, sums one launch of each), or
    None when there is no summary for it or the kernel sources changed since
    it was taken."""
    path = os.path.join(ROOT, "profiles", f"hbm_traffic_{workload}.json")
    try:
        with open(path) as f:
            rec = json.load(f)
    except (OSError, ValueError):
        return None
    if rec.get("sources_sha256") != kernel_sources_digest():
        return None
    ks = rec.get("kernels", {})
    base, _, srs = kernel.partition("<")
    names = [f"{base}<{sr}>" for sr in srs.rstrip(">").split("+")] if srs else [base]
    total = 0.0
    for nm in names:
        k = ks.get(nm) or (ks.get(base) if len(names) == 1 else None)
        if not k:
            return None
        total += k["read_bytes"] + k["write_bytes"]
    return int(round(total * launches))


# Counters of the L2-to-memory requests (TCC_EA0_*), one rocprofv3 pass for
# reads and one for writes (a pass holds at most four TCC counters).
READ_COUNTERS = ["TCC_EA0_RDREQ_sum", "TCC_EA0_RDREQ_32B_sum", "TCC_EA0_RDREQ_64B_sum", "TCC_EA0_RDREQ_128B_sum"]
WRITE_COUNTERS = ["TCC_EA0_WRREQ_sum", "TCC_EA0_WRREQ_64B_sum"]


def request_bytes(c):
    """HBM bytes of one dispatch from its request counts by size: read
    requests of 32, 64 and 128 bytes (any remainder of RDREQ counted as 64),
    write requests of 64 bytes (WRREQ_64B) and 32 bytes (the rest)."""
    r, r32, r64, r128 = (c["TCC_EA0_RDREQ_sum"], c["TCC_EA0_RDREQ_32B_sum"], c["TCC_EA0_RDREQ_64B_sum"],
                         c["TCC_EA0_RDREQ_128B_sum"])
    w, w64 = c["TCC_EA0_WRREQ_sum"], c["TCC_EA0_WRREQ_64B_sum"]
    rest = max(0.0, r - r32 - r64 - r128)
    return 32 * r32 + 64 * (r64 + rest) + 128 * r128, 64 * w64 + 32 * (w - w64)


def _counter_dispatches(dirs, short):
    """Per kernel (short name), its dispatches in launch order, each a dict of
    counter values plus 'ms', from the rocprofv3 counter-collection CSVs
    under ``dirs`` (one profiled run per directory)."""
    import csv
    import glob
    out = {}
    for d in dirs:
        per = {}
        for path in glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True):
            with open(path) as f:
                for r in csv.DictReader(f):
                    k = short(r["Kernel_Name"])
                    if k is None:
                        continue
                    e = per.setdefault(k, {}).setdefault(int(r["Dispatch_Id"]), {})
                    e[r["Counter_Name"]] = float(r["Counter_Value"])
                    e["ms"] = (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e6
        for k, ds in per.items():
            lst = [ds[i] for i in sorted(ds)]
            prev = out.setdefault(k, [])
            if not prev:
                prev.extend(dict(x) for x in lst)
            else:  # the same dispatches in the other pass: merge counters in launch order
                for x, y in zip(prev, lst):
                    x.update({c: v for c, v in y.items() if c != "ms"})
    return out


def _mean_counters(dispatches):
    keys = set().union(*[d.keys() for d in dispatches])
    return {c: float(np.mean([d[c] for d in dispatches if c in d])) for c in keys}


def _short_kernel_name(name):
    """k_rank_num<min_plus_i32> style names for the library's kernels, the
    calibration kernels by role, None for others."""
    sr = {"SrMinPlusI32": "min_plus_i32", "SrPattern": "or_and_bool", "SrOrAndBool": "or_and_bool",
          "SrPlusTimesF32": "plus_times_f32", "SrPlusTimesF64": "plus_times_f64", "SrMinPlusF32": "min_plus_f32",
          "SrMaxTimesF64": "max_times_f64", "SrMaxTimesF32": "max_times_f32"}
    if "spg::" in name:
        base = name.split("spg::", 1)[1].split("(")[0].split("<")[0].strip()
        for tag, nm in sr.items():
            if tag in name:
                fixed = base == "k_rank_num" and ", true>" in name
                return f"{base}{'_fixed' if fixed else ''}<{nm}>"
        return base
    low = name.lower()
    if "neg" in low:
        return "calib_stream"
    if "gather" in low or "index" in low:
        return "calib_gather"
    return None


CALIB_WIDTHS = (32, 64, 128, 4096)


def calib_rows(width):
    """Rows gathered per dispatch: 2^22, at most 1 GiB of them."""
    return min(1 << 22, (1 << 30) // width)


def calib_known():
    """Bytes per dispatch of the calibration kernels (run_calib): what they
    must move, each gathered row read once with its int64 id."""
    n = (1 << 30) // 4
    known = {"calib_stream": {"read_bytes": 4 * n, "write_bytes": 4 * n}}
    for w in CALIB_WIDTHS:
        known[f"calib_gather{w}"] = {"read_bytes": calib_rows(w) * (w + 8), "write_bytes": calib_rows(w) * w}
    return known


def run_counters(args):
    """Summary of two rocprofv3 counter runs of a workload (READ_COUNTERS,
    then WRITE_COUNTERS) and of the same two runs over the calibration
    workload: bytes per dispatch from request sizes, checked on the
    calibration kernels against their known bytes."""
    dirs = [d for d in args.counter_dirs.split(",") if d]
    if len(dirs) != 4:
        raise SystemExit("--counter-dirs needs: workload read dir, workload write dir, calib read dir, calib write dir")
    need = READ_COUNTERS + WRITE_COUNTERS
    kernels = {}
    for k, ds in _counter_dispatches(dirs[:2], _short_kernel_name).items():
        c = _mean_counters(ds)
        if not all(x in c for x in need):
            continue
        rb, wb = request_bytes(c)
        kernels[k] = {"read_bytes": rb, "write_bytes": wb, "avg_ms": round(c["ms"], 3), "dispatches": len(ds),
                      **{x: c[x] for x in need}}
    known = calib_known()
    calib = {}
    cal = _counter_dispatches(dirs[2:], _short_kernel_name)
    groups = {"calib_stream": cal.get("calib_stream", [])}
    g = cal.get("calib_gather", [])
    per = len(g) // len(CALIB_WIDTHS) if g else 0
    for j, w in enumerate(CALIB_WIDTHS):
        groups[f"calib_gather{w}"] = g[j * per:(j + 1) * per]
    for k, ds in groups.items():
        if not ds:
            continue
        c = _mean_counters(ds)
        if not all(x in c for x in need):
            continue
        rb, wb = request_bytes(c)
        calib[k] = {"read_bytes": rb, "write_bytes": wb,
                    "read_ratio": round(rb / known[k]["read_bytes"], 4),
                    "write_ratio": round(wb / known[k]["write_bytes"], 4), **{x: c[x] for x in need}}
    rec = {"workload": args.counter_workload, "command": args.counter_command,
           "sources_sha256": kernel_sources_digest(),
           "bytes": "read 32*RDREQ_32B + 64*RDREQ_64B + 128*RDREQ_128B (+ 64 per other RDREQ); "
                    "write 64*WRREQ_64B + 32*(WRREQ - WRREQ_64B); per dispatch, mean over dispatches",
           "calibration_known": known, "calibration_measured": calib, "kernels": kernels}
    if args.counter_out:
        with open(args.counter_out, "w") as f:
            json.dump(rec, f, indent=1)
    return rec


def run_calib(args):
    """Calibration kernels of known HBM bytes for the counter summaries: a
    streaming float32 negation of 1 GiB (reads 1 GiB, writes 1 GiB), then row
    gathers from a 4 GiB table (far larger than the caches) of random rows of
    32, 64, 128 and 4096 bytes (2^22 rows, at most 1 GiB of them; reads the
    rows and the int64 row ids, writes the rows), each launched ``--steps``
    times."""
    import torch
    dev = torch.device("cuda:0")
    reps = max(1, args.steps)
    n = (1 << 30) // 4
    x = torch.ones(n, dtype=torch.float32, device=dev)
    y = torch.empty_like(x)
    torch.cuda.synchronize()
    for _ in range(reps):
        torch.neg(x, out=y)
    torch.cuda.synchronize()
    del x, y
    g = torch.Generator(device="cpu").manual_seed(5)
    for width in CALIB_WIDTHS:
        cols = width // 4
        table = torch.zeros(((4 << 30) // width, cols), dtype=torch.float32, device=dev)
        ids = torch.randint(0, table.shape[0], (calib_rows(width),), generator=g).to(dev)
        out = torch.empty((calib_rows(width), cols), dtype=torch.float32, device=dev)
        torch.cuda.synchronize()
        for _ in range(reps):
            torch.index_select(table, 0, ids, out=out)
        torch.cuda.synchronize()
        del table, ids, out
        torch.cuda.empty_cache()
    return {"workload": "calibration kernels of known bytes", "reps": reps, "known": calib_known()}


def alg_bytes_dense(A, nnz_dense_rows_A, ndense_rows, nnz_c_dense, s_in, s_out, symbolic):
    """Algorithmic HBM bytes of one dense-accumulator launch: read the row
    list, the A rows it covers and B once; write C's entries (numeric) or the
    row sizes (symbolic)."""
    n = A.nrows
    b_once = 8 * (n + 1) + (4 + s_in) * A.nnz
    a_rows = 16 * ndense_rows + 4 * ndense_rows + (4 + s_in) * nnz_dense_rows_A
    if symbolic:
        return b_once - s_in * A.nnz + a_rows - s_in * nnz_dense_rows_A + 8 * ndense_rows
    return b_once + a_rows + 8 * ndense_rows + (4 + s_out) * nnz_c_dense


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU; --gpus {args.gpus} is not supported "
              f"(the product is a single-GPU kernel path)", file=sys.stderr)
        sys.exit(2)
    run = {"rmat": run_rmat, "er": run_er, "mcl": run_mcl, "batched": run_batched,
           "served": run_served, "merge": run_merge, "outbatch": run_outbatch, "calib": run_calib,
           "counters": run_counters}[args.workload]
    out = run(args)
    print(json.dumps(out), flush=True)


def base_record(args, value, unit, ms_per_step, dtype, config, higher=True):
    return {"metric": METRIC, "value": value, "unit": unit, "n_gpus": 1, "steps": args.steps,
            "warmup": args.warmup, "ms_per_step": round(ms_per_step, 3), "higher_is_better": higher,
            "scaling": "weak", "vs_baseline": None, "dtype": dtype, "data": "synthetic", "config": config}


# Numeric bins of the library's row classes (spg_launch.h): hash classes
# 1..14 (15 holds the rows whose kept bitmap is expanded), expand-sort-compress
# classes from 55 on.
HASH_BINS_END = 15
ESC_BIN_BASE = 55


def row_flops(H):
    """Products per output slice of H*H (oriented CSR arrays), from the host
    copy of the operand (bookkeeping for the algorithmic bytes only)."""
    deg = np.diff(H.ptr)
    return np.bincount(np.repeat(np.arange(deg.size), deg), weights=deg[H.idx].astype(np.float64),
                       minlength=deg.size), deg


def dominant_kernel(H, phase, rownnz, p, s_in, s_out, sr):
    """The longest launch of one product H*H among the library's kernels,
    with its algorithmic HBM bytes: A's rows it covers and B read once, C's
    entries of those rows written once (numeric) or the row sizes
    (symbolic).  phase: the plan's phase times; rownnz: entries per slice."""
    fl, deg = row_flops(H)
    sym_dense_rows = fl > p.hash_max_flops()
    hmn = p.hash_max_nnz()
    ranked = phase.get("num_rank", 0.0) > 0
    # pattern-only products expand the rows whose symbolic bitmap was kept
    # (at least one product per bitmap word; the budget is taken as enough)
    kept = sym_dense_rows & (fl >= -(-H.ncols // 32)) if sr == "or_and_bool" and not ranked \
        else np.zeros_like(sym_dense_rows)
    o = p.options()
    esc_rows = (rownnz > 0) & ~kept & (fl <= max(0, o.esc_max_flops)) & (16 * fl <= o.esc_ratio_x16 * rownnz)
    heavy = sym_dense_rows & (rownnz > hmn) & ~esc_rows
    fixed_rows = heavy & (rownnz * p.rank_dense_div() >= H.ncols)
    rank_rows = heavy & ~fixed_rows if ranked else np.zeros_like(sym_dense_rows)
    num_dense_rows = (rownnz > hmn) & ~rank_rows & ~kept & ~esc_rows
    hash_rows = (rownnz > 0) & (rownnz <= hmn) & ~kept & ~esc_rows

    def num_bytes(rows):
        return alg_bytes_dense(H, int(deg[rows].sum()), int(rows.sum()), int(rownnz[rows].sum()), s_in, s_out,
                               False)
    cands = {
        "k_expand_rows": (phase.get("num_expand", 0.0), num_bytes(kept)),
        "k_hash_num": (phase.get("num_hash", 0.0), num_bytes(hash_rows)),
        "k_esc_num": (phase.get("num_esc", 0.0), num_bytes(esc_rows)),
        "k_dense_num": (phase.get("num_dense", 0.0), num_bytes(num_dense_rows)),
        "k_rank_num": (phase.get("num_rank", 0.0), num_bytes(rank_rows)),
        "k_dense_sym": (phase.get("sym_dense", 0.0), alg_bytes_dense(
            H, int(deg[sym_dense_rows].sum()), int(sym_dense_rows.sum()), 0, s_in, 0, True)),
        "k_hash_sym": (phase.get("sym_hash", 0.0), alg_bytes_dense(
            H, int(deg[~sym_dense_rows].sum()), int((~sym_dense_rows).sum()), 0, s_in, 0, True)),
    }
    # launches per phase: one per non-empty class of the hash and ESC kernels
    sym_bins, num_bins = p.bins()
    launches = {"k_hash_num": sum(1 for c in range(1, HASH_BINS_END) if num_bins[c]),
                "k_esc_num": sum(1 for c in range(ESC_BIN_BASE, len(num_bins)) if num_bins[c]),
                "k_hash_sym": sum(1 for c in range(1, HASH_BINS_END + 1) if sym_bins[c])}
    dom = None
    for name, (ms, by) in cands.items():
        if ms > 0 and (dom is None or ms > dom["ms"]):
            dom = {"kernel": name, "semiring": sr, "ms": ms, "bytes": by, "launches": max(1, launches.get(name, 1))}
    return dom


def roofline_record(dom, workload):
    achieved = dom["bytes"] / (dom["ms"] * 1e-3) / 1e9
    name = f"{dom['kernel']}<{dom['semiring']}>"
    rec = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
           "frac": round(achieved / HBM_PEAK_GBS, 4),
           "traffic": measured_traffic(name, workload, dom.get("launches", 1)),
           "kernel": name, "kernel_ms": round(dom["ms"], 3), "alg_bytes": int(dom["bytes"])}
    if dom.get("launches", 1) > 1:
        rec["launches"] = dom["launches"]  # one per accumulator class, timed together
    return rec


def run_rmat(args):
    import torch

    import spgen
    from paper_2106_14402_amd import binding as B
    from paper_2106_14402_amd import spgemm as S

    dev = torch.device("cuda:0")
    t0 = time.time()
    log(f"[bench] generating R-MAT scale {args.scale} ...")
    H = spgen.rmat_graph(args.scale, 16, spgen.rng_for(1), symmetric=True, weights="i32")
    log(f"[bench] generated n={H.nrows} nnz={H.nnz} in {time.time() - t0:.1f}s")
    Ad = S.to_device(H, dev)
    Apat = S.DeviceMatrix(Ad.nrows, Ad.ncols, "csr", Ad.ptr, Ad.idx, None)
    semirings = args.semirings.split(",")
    mats = {"or_and_bool": Apat, "min_plus_i32": Ad}
    s_in = {"or_and_bool": 0, "min_plus_i32": 4}
    s_out = {"or_and_bool": 0, "min_plus_i32": 4}
    extra = {k: int(v) for k, v in (o.split("=") for o in args.opt)}
    opts = {"or_and_bool": B.make_options(timing=1, bitmap_mib=args.bitmap_mib, **extra),
            "min_plus_i32": B.make_options(timing=1, bitmap_mib=args.bitmap_mib_valued, **extra)}
    prods = {sr: S.Product(mats[sr], mats[sr], sr, opts[sr]) for sr in semirings}
    c_ptr = torch.empty(H.nrows + 1, dtype=torch.int64, device=dev)

    # sizes (one symbolic pass, outside timing) and output buffers
    nnz_c, flops = {}, {}
    for sr, p in prods.items():
        nnz_c[sr] = p.symbolic(c_ptr)
        flops[sr] = p.stats()[0]
        log(f"[bench] {sr}: flops={flops[sr]} nnz(C)={nnz_c[sr]}")
    max_nnz = max(nnz_c.values())
    buf_idx = torch.empty(max_nnz, dtype=torch.int32, device=dev)
    buf_val = torch.empty(max_nnz if "min_plus_i32" in prods else 0, dtype=torch.int32, device=dev)
    log(f"[bench] output buffers {(buf_idx.numel() + buf_val.numel()) * 4 / 1e9:.1f} GB; "
        f"free {torch.cuda.mem_get_info()[0] / 1e9:.1f} GB")

    def step(record):
        for sr, p in prods.items():
            nz = p.symbolic(c_ptr)
            p.numeric(c_idx=buf_idx[:nz], c_val=None if sr == "or_and_bool" else buf_val[:nz])
            if record is not None:
                record.setdefault(sr, []).append(p.timings())

    for _ in range(args.warmup):
        step(None)
    torch.cuda.synchronize()
    record = {}
    t1 = time.perf_counter()
    for _ in range(args.steps):
        step(record)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t1
    ms_per_step = elapsed * 1e3 / args.steps
    total_flops = sum(flops.values())
    gflops = 2.0 * total_flops * args.steps / elapsed / 1e9
    log(f"[bench] {ms_per_step:.2f} ms/step, {gflops:.1f} GFLOP/s")

    # phase means and the dominant kernel
    phase_ms = {sr: {k: float(np.mean([r[k] for r in recs])) for k in recs[0]} for sr, recs in record.items()}
    dom = None
    for sr, p in prods.items():
        p.symbolic(c_ptr)
        rownnz = torch.diff(c_ptr).cpu().numpy()
        d = dominant_kernel(H, phase_ms[sr], rownnz, p, s_in[sr], s_out[sr], sr)
        if dom is None or d["ms"] > dom["ms"]:
            dom = d
    roofline = roofline_record(dom, f"rmat{args.scale}")
    # whole-step compulsory bytes (two-phase, B cached): per product
    bmin = 0
    for sr in prods:
        n = H.nrows
        pat = 8 * (n + 1) + 4 * H.nnz
        bmin += 3 * pat + 2 * pat + 2 * s_in[sr] * H.nnz + (4 + s_out[sr]) * nnz_c[sr] + 8 * (n + 1) + 24 * n

    out = {
        "metric": METRIC,
        "value": round(gflops, 2),
        "unit": "GFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "+".join({"or_and_bool": "bool(pattern)", "min_plus_i32": "int32"}[s] for s in prods),
        "data": "synthetic",
        "config": {
            "workload": f"R-MAT scale {args.scale} squared: (OR,AND) pattern and (min,+) int32",
            "n": H.nrows, "edge_factor": 16, "rmat": [0.57, 0.19, 0.19, 0.05], "symmetrized": True,
            "nnz_A": H.nnz, "flops": {k: int(v) for k, v in flops.items()},
            "nnz_C": {k: int(v) for k, v in nnz_c.items()},
        },
        "roofline": roofline,
        "bmin_gbs": round(bmin / (ms_per_step * 1e-3) / 1e9, 1),
        "phase_ms": {sr: {k: round(v, 3) for k, v in d.items() if v > 0} for sr, d in phase_ms.items()},
    }
    for p in prods.values():
        p.close()
    del buf_idx, buf_val
    torch.cuda.empty_cache()

    if args.cpu_seconds > 0:
        out["cpu_baseline"] = cpu_baseline(H, list(prods), args.cpu_seconds)
    return out


def cpu_baseline(H, semirings, target_s):
    """The oracle on a seeded row sample of the same workload, all host
    threads; rate = 2 x sample products / time."""
    import oracle

    nthreads = int(os.environ.get("OMP_NUM_THREADS", "0")) or os.cpu_count()
    rng = np.random.default_rng(7)
    fl = oracle.flops(H, H)
    order = rng.permutation(H.nrows)
    # probe the rate on a small sample, then size the timed sample
    probe = order[:256]
    t = time.perf_counter()
    for sr in semirings:
        oracle.spgemm(H if sr != "or_and_bool" else H.with_values(None), H if sr != "or_and_bool" else H.with_values(None),
                      sr, select=probe, nthreads=nthreads)
    dt = max(time.perf_counter() - t, 1e-3)
    rate = fl[probe].sum() * len(semirings) / dt
    want = rate * target_s / len(semirings)
    csum = np.cumsum(fl[order])
    nsel = int(np.searchsorted(csum, want)) + 1
    sel = np.sort(order[:max(nsel, 1)])
    t = time.perf_counter()
    for sr in semirings:
        M = H if sr != "or_and_bool" else H.with_values(None)
        oracle.spgemm(M, M, sr, select=sel, nthreads=nthreads)
    dt = time.perf_counter() - t
    sample_flops = int(fl[sel].sum()) * len(semirings)
    return {"value": round(2.0 * sample_flops / dt / 1e9, 4), "unit": "GFLOP/s", "cores": nthreads,
            "kind": "oracle",
            "sample": f"{sel.size} seeded random rows of {H.nrows} ({sample_flops} products over "
                      f"{len(semirings)} semirings, {dt:.1f} s)"}


def timed(fn, steps, warmup):
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    t = time.perf_counter()
    for _ in range(steps):
        fn()
    torch.cuda.synchronize()
    return (time.perf_counter() - t) * 1e3 / steps


def run_er(args):
    """Erdos-Renyi n=4096, 8 per row, (+,x) float64 (launch-latency bound)."""
    import torch

    import spgen
    from paper_2106_14402_amd import spgemm as S
    A = spgen.config_er()
    dA = S.to_device(A)
    p = S.Product(dA, dA, "plus_times_f64")
    nnz = p.symbolic()
    flops = p.stats()[0]
    c_idx = torch.empty(nnz, dtype=torch.int32, device="cuda")
    c_val = torch.empty(nnz, dtype=torch.float64, device="cuda")

    def step():
        p.symbolic(p.c_ptr)
        p.numeric(c_idx, c_val)
    ms = timed(step, args.steps, args.warmup)
    out = base_record(args, round(2.0 * flops / (ms * 1e-3) / 1e9, 3), "GFLOP/s", ms, "f64",
                      {"workload": "Erdos-Renyi n=4096, 8 per row, C=A*A over (+,x) float64",
                       "flops": flops, "nnz_C": nnz})
    out["us_per_product"] = round(ms * 1e3, 1)
    if args.cpu_seconds > 0:
        import oracle
        nthreads = int(os.environ.get("OMP_NUM_THREADS", "0")) or os.cpu_count()
        t = time.perf_counter()
        reps = 0
        while time.perf_counter() - t < min(args.cpu_seconds, 5):
            oracle.spgemm(A, A, "plus_times_f64", nthreads=nthreads)
            reps += 1
        dt = (time.perf_counter() - t) / reps
        out["cpu_baseline"] = {"value": round(2.0 * flops / dt / 1e9, 4), "unit": "GFLOP/s",
                               "cores": nthreads, "kind": "oracle",
                               "sample": f"whole product, mean of {reps} runs"}
    p.close()
    return out


def run_mcl(args):
    """Markov-clustering expansion: column-stochastic n=2^20 float32 CSC,
    C=A*A over (+,x) float32, then prune entries < 1e-4."""
    import torch

    import spgen
    from paper_2106_14402_amd import binding as B
    from paper_2106_14402_amd import spgemm as S
    t0 = time.time()
    A = spgen.config_mcl()
    log(f"[bench] MCL matrix n={A.ncols} nnz={A.nnz} in {time.time() - t0:.1f}s")
    dA = S.to_device(A)
    extra = {k: int(v) for k, v in (o.split("=") for o in args.opt)}
    p = S.Product(dA, dA, "plus_times_f32", B.make_options(timing=1, **extra))
    nnz = p.symbolic()
    flops = p.stats()[0]
    c_idx = torch.empty(nnz, dtype=torch.int32, device="cuda")
    c_val = torch.empty(nnz, dtype=torch.float32, device="cuda")
    state = {}

    def step():
        p.symbolic(p.c_ptr)
        C = p.numeric(c_idx, c_val)
        state["P"] = S.prune_f32(C, 1e-4)
    ms = timed(step, args.steps, args.warmup)
    kept = state["P"].nnz

    phase = {k: v for k, v in p.timings().items()}
    rownnz = torch.diff(p.c_ptr).cpu().numpy()

    def expansion():  # the product alone, without the prune
        p.symbolic(p.c_ptr)
        p.numeric(c_idx, c_val)
    ms_exp = timed(expansion, args.steps, 1)

    def iteration():  # the whole Markov-clustering iteration: expansion, prune, selection, inflation (r = 2)
        step()
        state["Q"] = S.select_f32(state["P"], args.select)
        S.inflate_f32(state["Q"], 2.0)
    ms_it = timed(iteration, max(1, args.steps // 2), 1)
    out = base_record(args, round(2.0 * flops / (ms * 1e-3) / 1e9, 2), "GFLOP/s", ms, "f32",
                      {"workload": "MCL expansion n=2^20, lognormal column degree mean 48 (sigma 1), "
                                   "column-stochastic float32 CSC, C=A*A over (+,x) float32, prune < 1e-4",
                       "n": A.ncols, "nnz_A": A.nnz, "flops": flops, "nnz_C": nnz, "nnz_pruned": kept,
                       "select": args.select, "nnz_selected": state["Q"].nnz})
    out["roofline"] = roofline_record(dominant_kernel(A, phase, rownnz, p, 4, 4, "plus_times_f32"), "mcl")
    out["phase_ms"] = {k: round(v, 3) for k, v in phase.items() if v > 0}
    out["expansion_ms"] = round(ms_exp, 3)
    out["iteration_ms"] = round(ms_it, 3)
    if args.cpu_seconds > 0:
        out["cpu_baseline"] = cpu_baseline_generic(A, "plus_times_f32", args.cpu_seconds)
    p.close()
    return out


def run_batched(args):
    """512 uneven products (ER / R-MAT, (+,x) float64 / (min,+) int32) in one
    batched plan, against one call per product writing into the same pooled
    outputs.  Two comparisons: the whole step (symbolic + numeric) and the
    numeric phase alone (the batched one replayed from its hipGraph)."""
    import torch

    import spgen
    from paper_2106_14402_amd import batch as BT
    from paper_2106_14402_amd import spgemm as S
    t0 = time.time()
    items = spgen.batch_mix(nprod=args.nprod)
    mats = [S.to_device(it.A) for it in items]
    srs = [it.semiring for it in items]
    log(f"[bench] {len(items)} products generated in {time.time() - t0:.1f}s")
    from paper_2106_14402_amd import autotune as AT
    cache = os.path.join(ROOT, "gpurun_out", "autotune.json") if args.autotune_cache is None else args.autotune_cache
    if args.batch_knobs:
        # knob values given on the command line (e.g. a profiled run that must
        # not include the tuner's trials)
        knobs = {k: int(v) for k, v in (kv.split("=") for kv in args.batch_knobs.split(","))}
        tuning = {"knobs": knobs, "ms": None, "default_ms": None, "from_cache": False, "given": True}
    else:
        tuning = AT.tune_batch(mats, mats, srs, cache, log=log)
    log(f"[bench] autotuned {tuning}")
    bopt = AT.make_options(tuning["knobs"])
    bopt.timing = 1
    bp = BT.BatchProduct(mats, mats, srs, bopt)
    bp.symbolic()
    bp.allocate()
    flops = bp.stats()[0]
    record = []

    def batched_full():
        bp.symbolic()
        bp.numeric()
        record.append(bp.timings())
    ms_b = timed(batched_full, args.steps, args.warmup)
    phase_ms = {k: float(np.mean([r[k] for r in record[args.warmup:]])) for k in record[0]}
    roofline = roofline_record(batched_dominant(items, bp, phase_ms, tuning["knobs"]), "batched")
    bp.capture()
    ms_br = timed(bp.replay, args.steps, args.warmup)
    singles = [S.Product(m, m, sr) for m, sr in zip(mats, srs)]
    vb = BT.VAL_BYTES
    outs = []
    for b, pr in enumerate(singles):
        nz = bp.c_nnz[b]
        idx = bp.c_idx[bp.idx_off[b]:bp.idx_off[b] + nz]
        raw = bp.c_val[bp.val_off[b]:bp.val_off[b] + nz * vb[srs[b]]]
        outs.append((bp.c_ptr[bp.pool_off[b]:bp.pool_off[b + 1]], idx,
                     raw.view(S.OUT_DTYPE[srs[b]]) if nz else None))

    def one_by_one_full():
        for pr, (cp, idx, val) in zip(singles, outs):
            pr.symbolic(cp)
            pr.numeric(idx, val)

    def one_by_one_numeric():
        for pr, (_, idx, val) in zip(singles, outs):
            pr.numeric(idx, val)
    ms_s = timed(one_by_one_full, max(1, args.steps // 2), 1)
    ms_sn = timed(one_by_one_numeric, max(1, args.steps // 2), 1)
    for pr in singles:
        pr.close()
    out = base_record(args, round(2.0 * flops / (ms_b * 1e-3) / 1e9, 2), "GFLOP/s", ms_b, "f64+int32",
                      {"workload": f"{len(items)} uneven products: n log-uniform in [1K,64K], degree 4-32, "
                                   "half Erdos-Renyi / half R-MAT, (+,x) float64 and (min,+) int32",
                       "flops": flops, "nnz_C": int(sum(bp.c_nnz))})
    out["batched"] = {"full_step_ms": round(ms_b, 3), "numeric_graph_replay_ms": round(ms_br, 3)}
    out["one_call_per_product"] = {"full_step_ms": round(ms_s, 3), "numeric_ms": round(ms_sn, 3)}
    out["speedup"] = {"full_step": round(ms_s / ms_b, 3), "numeric": round(ms_sn / ms_br, 3)}
    out["autotune"] = {"knobs": tuning["knobs"], "tuned_ms": tuning["ms"], "default_ms": tuning["default_ms"],
                       "from_cache": tuning["from_cache"], "given": bool(tuning.get("given"))}
    out["roofline"] = roofline
    out["phase_ms"] = {k: round(v, 3) for k, v in phase_ms.items()}
    bp.close()
    return out


def batched_dominant(items, bp, phase_ms, knobs):
    """The longest phase of a batched step (its launches cover every
    product's rows of one accumulator family) with its algorithmic bytes,
    summed over the products: for each, its covered A rows and B read once,
    C's entries of those rows written once (numeric) or the row sizes
    (symbolic)."""
    hmn = int(knobs.get("hash_max_nnz", 2048))
    hmf = int(knobs.get("hash_max_flops", 8192))
    esc_max = int(knobs.get("esc_max_flops", 8192))  # the batch's semirings all hold the 8192 class
    esc_ratio = int(knobs.get("esc_ratio_x16", 20))  # the batched plan's default
    byts = {k: 0 for k in phase_ms}
    for b, it in enumerate(items):
        s_io = 8 if it.semiring == "plus_times_f64" else 4
        fl, deg = row_flops(it.A)
        rownnz = np.diff(bp.c_ptr[bp.pool_off[b]:bp.pool_off[b + 1]].cpu().numpy())
        esc = (rownnz > 0) & (fl <= esc_max) & (16 * fl <= esc_ratio * rownnz)
        dense = (rownnz > hmn) & ~esc
        hashed = (rownnz > 0) & ~dense & ~esc
        heavy = fl > hmf
        light = (fl > 0) & ~heavy
        for name, rows, sym in (("num_dense", dense, False), ("num_hash", hashed, False), ("num_esc", esc, False),
                                ("sym_dense", heavy, True), ("sym_hash", light, True)):
            if rows.any():
                byts[name] += alg_bytes_dense(it.A, int(deg[rows].sum()), int(rows.sum()),
                                              int(rownnz[rows].sum()), s_io, s_io, sym)
    kern = {"num_dense": "k_dense_num_b", "num_hash": "k_hash_num_b", "num_esc": "k_esc_num_b",
            "sym_dense": "k_dense_sym_b", "sym_hash": "k_hash_sym_b"}
    name = max(phase_ms, key=lambda k: phase_ms[k])
    return {"kernel": kern[name], "semiring": "plus_times_f64+min_plus_i32", "ms": phase_ms[name],
            "bytes": byts[name]}


def run_served(args):
    """Resident R-MAT scale-22 adjacency (directed, pattern only); Poisson
    streams of frontier requests F' = A^T F over (OR,AND) at three rates,
    served with continuous batching and with one call per request."""
    import numpy as np

    import spgen
    from paper_2106_14402_amd import serve as SV
    t0 = time.time()
    A = spgen.config_served_graph()
    log(f"[bench] served graph n={A.nrows} nnz={A.nnz} in {time.time() - t0:.1f}s")
    g = SV.ResidentGraph(A)
    rng = spgen.rng_for(4, 7)
    # one-at-a-time service rate mu1 (back-to-back requests, one call each)
    probe = spgen.request_stream(A.nrows, 300, 1e9, rng)
    single = SV.FrontierServer(g, workers=1, max_batch_requests=1)
    res = single.serve(probe)
    mu1 = SV.latency_summary(res)["req_per_s"]
    log(f"[bench] one call per request: {mu1:.0f} req/s")
    rates = {}
    # below, near and above the one-call rate, then every request at once
    # (closed loop: the sustained throughput of each mode)
    for frac in (0.3, 0.6, 0.9, 1.5, 3.0, None):
        lam = 1e9 if frac is None else frac * mu1
        sub = 99 if frac is None else int(frac * 10)
        reqs = spgen.request_stream(A.nrows, args.requests, lam, spgen.rng_for(4, sub))
        r_batch = SV.latency_summary(SV.FrontierServer(g, workers=3).serve(reqs))
        r_single = SV.latency_summary(SV.FrontierServer(g, workers=1, max_batch_requests=1).serve(reqs))
        key = "saturation" if frac is None else f"{frac:.1f}mu1"
        rates[key] = {"rate_req_s": None if frac is None else round(lam, 1), "batched": r_batch,
                      "one_call": r_single}
        log(f"[bench] {key}: batched {r_batch['req_per_s']:.0f} req/s p50 {r_batch['p50_ms']:.2f} "
            f"p99 {r_batch['p99_ms']:.2f} | single {r_single['req_per_s']:.0f} req/s "
            f"p50 {r_single['p50_ms']:.2f} p99 {r_single['p99_ms']:.2f}")
    top = rates["0.9mu1"]["batched"]
    out = base_record(args, round(top["p99_ms"], 3), "ms (p99 at 0.9 mu1)", top["mean_ms"], "bool(pattern)",
                      {"workload": "served frontier expansion on resident R-MAT scale 22 (edge factor 16, "
                                   "directed), k log-uniform in [1,1024], 1-64 sources per column",
                       "n": A.nrows, "nnz_A": A.nnz, "requests_per_rate": args.requests}, higher=False)
    out["mu1_req_s"] = round(mu1, 1)
    out["max_sustained_req_s"] = {"batched": round(rates["saturation"]["batched"]["req_per_s"], 1),
                                  "one_call": round(rates["saturation"]["one_call"]["req_per_s"], 1)}
    out["rates"] = rates
    return out


def run_merge(args):
    """Merge of SUMMA partial products: R-MAT scale 18 (symmetrised, int32
    weights) squared over (min,+) with the inner dimension cut into 4 equal
    blocks; the 4 partial products A(:,K_t) A(K_t,:) are formed once, and a
    step is their semiring sum (symbolic + numeric).  Reported as HBM GB/s of
    the algorithmic bytes (read every part once, write C once)."""
    import torch

    import spgen
    from paper_2106_14402_amd import spgemm as S
    t0 = time.time()
    H = spgen.rmat_graph(18, 16, spgen.rng_for(1, 18), symmetric=True, weights="i32")
    log(f"[bench] R-MAT scale 18 nnz={H.nnz} in {time.time() - t0:.1f}s")
    k, n = 4, H.nrows
    cuts = [n * t // k for t in range(k + 1)]
    rows = np.repeat(np.arange(n), np.diff(H.ptr))
    parts = []
    for lo, hi in zip(cuts[:-1], cuts[1:]):
        kc = (H.idx >= lo) & (H.idx < hi)
        kr = (rows >= lo) & (rows < hi)
        Ac = spgen.from_pairs(n, n, rows[kc], H.idx[kc], H.val[kc])
        Br = spgen.from_pairs(n, n, rows[kr], H.idx[kr], H.val[kr])
        parts.append(S.spgemm(S.to_device(Ac), S.to_device(Br), "min_plus_i32"))
    torch.cuda.synchronize()
    P = S.stack(parts)
    in_nnz = int(P.nnz)
    from paper_2106_14402_amd import binding as B
    extra = {kk: int(v) for kk, v in (o.split("=") for o in args.opt)}
    p = S.SumPlan(P, k, "min_plus_i32", B.make_options(timing=1, **extra))
    nnz = p.symbolic()
    c_idx = torch.empty(nnz, dtype=torch.int32, device="cuda")
    c_val = torch.empty(nnz, dtype=torch.int32, device="cuda")

    def step():
        p.symbolic(p.c_ptr)
        p.numeric(c_idx, c_val)
    ms = timed(step, args.steps, args.warmup)
    alg = 8 * in_nnz + 8 * (k * n + 1) + 8 * nnz + 8 * (n + 1)
    gbs = alg / (ms * 1e-3) / 1e9
    out = base_record(args, round(gbs, 1), "GB/s", ms, "int32",
                      {"workload": "merge of 4 SUMMA partial products of R-MAT scale 18 squared over (min,+) int32",
                       "n": n, "parts": k, "entries_in": in_nnz, "nnz_C": nnz})
    out["roofline"] = {"bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                       "frac": round(gbs / HBM_PEAK_GBS, 4), "traffic": None, "kernel": "whole merge step",
                       "alg_bytes": alg}
    out["phase_ms"] = {kk: round(v, 3) for kk, v in p.timings().items() if v > 0}
    if args.cpu_seconds > 0:
        import oracle
        nthreads = int(os.environ.get("OMP_NUM_THREADS", "0")) or os.cpu_count()
        hp = [(x.ptr.cpu().numpy(), x.idx.cpu().numpy(), x.val.cpu().numpy()) for x in parts]
        sel = np.sort(np.random.default_rng(7).choice(n, size=min(n, 20000), replace=False))
        sub = []
        for pp, pi, pv in hp:
            cnt = pp[sel + 1] - pp[sel]
            ptr = np.concatenate([[0], np.cumsum(cnt)]).astype(np.int64)
            take = np.concatenate([np.arange(pp[r], pp[r + 1]) for r in sel])
            sub.append(spgen.SparseMatrix(sel.size, n, "csr", ptr, pi[take], pv[take]))
        t = time.perf_counter()
        res = oracle.sum_parts(sub, "min_plus_i32", nthreads=nthreads)
        dt = time.perf_counter() - t
        sub_alg = 8 * sum(x.nnz for x in sub) + 8 * (k * sel.size + 1) + 8 * int(res[0][-1]) + 8 * (sel.size + 1)
        out["cpu_baseline"] = {"value": round(sub_alg / dt / 1e9, 3), "unit": "GB/s", "cores": nthreads,
                               "kind": "oracle", "sample": f"{sel.size} seeded random rows of {n} ({dt:.1f} s)"}
    p.close()
    return out


def run_outbatch(args):
    """Output formed in batches: R-MAT scale 20 (symmetrised, int32 weights)
    squared over (min,+), with an output budget of nnz(C) / 4 entries (the
    paper forms its largest product in 4 batches).  A step is the symbolic
    phase, the split of the slices into ranges that fit the budget (from the
    offsets, on the host), and the numeric phase of each range into the same
    two buffers of budget size.  The same product in one call is timed
    beside it."""
    import torch

    import spgen
    from paper_2106_14402_amd import binding as B
    from paper_2106_14402_amd import spgemm as S
    t0 = time.time()
    H = spgen.rmat_graph(args.scale, 16, spgen.rng_for(1), symmetric=True, weights="i32")
    log(f"[bench] R-MAT scale {args.scale} nnz={H.nnz} in {time.time() - t0:.1f}s")
    extra = {k: int(v) for k, v in (o.split("=") for o in args.opt)}
    dA = S.to_device(H)
    p = S.Product(dA, dA, "min_plus_i32", B.make_options(bitmap_mib=args.bitmap_mib_valued, **extra))
    nnz = p.symbolic()
    flops = p.stats()[0]
    budget = -(-nnz // args.batches)
    ranges = p.row_batches(budget)
    cap = max(int(p.c_ptr[re] - p.c_ptr[rb]) for rb, re in ranges)
    idx = torch.empty(cap, dtype=torch.int32, device="cuda")
    val = torch.empty(cap, dtype=torch.int32, device="cuda")
    log(f"[bench] nnz(C)={nnz} budget={budget} -> {len(ranges)} ranges, largest {cap}")

    def step():
        p.symbolic(p.c_ptr)
        for rb, re in p.row_batches(budget):
            p.numeric_rows(rb, re, idx, val)
    ms = timed(step, args.steps, args.warmup)
    del idx, val
    full_idx = torch.empty(nnz, dtype=torch.int32, device="cuda")
    full_val = torch.empty(nnz, dtype=torch.int32, device="cuda")

    def single():
        p.symbolic(p.c_ptr)
        p.numeric(full_idx, full_val)
    ms_single = timed(single, args.steps, args.warmup)
    out = base_record(args, round(2.0 * flops / (ms * 1e-3) / 1e9, 2), "GFLOP/s", ms, "int32",
                      {"workload": f"R-MAT scale {args.scale} squared over (min,+) int32, output formed in batches "
                                   f"of at most nnz(C)/{args.batches} entries",
                       "flops": flops, "nnz_C": nnz, "batches": len(ranges), "budget_entries": budget})
    out["output_buffer_bytes"] = 8 * cap
    out["single_call_output_bytes"] = 8 * nnz
    out["single_call_ms"] = round(ms_single, 3)
    out["batched_over_single"] = round(ms / ms_single, 4)
    if args.cpu_seconds > 0:
        out["cpu_baseline"] = cpu_baseline_generic(H, "min_plus_i32", args.cpu_seconds)
    p.close()
    return out


def cpu_baseline_generic(A, semiring, target_s):
    """The oracle on a seeded slice sample of a square product."""
    import oracle

    nthreads = int(os.environ.get("OMP_NUM_THREADS", "0")) or os.cpu_count()
    fl = oracle.flops(A, A)
    order = np.random.default_rng(7).permutation(fl.size)
    probe = order[:256]
    t = time.perf_counter()
    oracle.spgemm(A, A, semiring, select=probe, nthreads=nthreads)
    rate = fl[probe].sum() / max(time.perf_counter() - t, 1e-3)
    nsel = int(np.searchsorted(np.cumsum(fl[order]), rate * target_s)) + 1
    sel = np.sort(order[:nsel])
    t = time.perf_counter()
    oracle.spgemm(A, A, semiring, select=sel, nthreads=nthreads)
    dt = time.perf_counter() - t
    return {"value": round(2.0 * int(fl[sel].sum()) / dt / 1e9, 4), "unit": "GFLOP/s", "cores": nthreads,
            "kind": "oracle", "sample": f"{sel.size} seeded random slices of {fl.size} ({dt:.1f} s)"}


if __name__ == "__main__":
    main()
