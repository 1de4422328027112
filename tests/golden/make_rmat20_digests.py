"""Writes the block digests of the R-MAT scale-20 squares for the full-output
parity test (tests/golden/rmat20_digests.json).

Calls the oracle only: every slice of C = A*A (paper Sec. 3.1) is formed by
the oracle's Gustavson product, hashed and dropped (C is never held), for
(OR,AND) on the pattern and (min,+) with int32 weights, on the seeded
scale-20 workload the benchmark squares.  Runs on the host cores; about an
hour on 8 cores.

    python tests/golden/make_rmat20_digests.py [--scale 20] [--out PATH]
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import spgen  # noqa: E402

BLOCK = 1024


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--scale", type=int, default=20)
    ap.add_argument("--rows-per-call", type=int, default=1 << 16)
    ap.add_argument("--out", default=None)
    args = ap.parse_args()
    out = args.out or os.path.join(os.path.dirname(os.path.abspath(__file__)), f"rmat{args.scale}_digests.json")
    H = spgen.rmat_graph(args.scale, 16, spgen.rng_for(1), symmetric=True, weights="i32")
    n = H.nrows
    rec = {"workload": f"R-MAT scale {args.scale}, edge factor 16, a=.57 b=.19 c=.19 d=.05, symmetrised, "
                       "no loops or duplicates, seeded relabelling; int32 weights U[1,255] (spgen.rmat_graph "
                       "with spgen.rng_for(1)); C = A*A",
           "nnz_A": H.nnz, "nrows": n, "block": BLOCK,
           "digest": "slice: sum over entries t of mix64(mix64((t<<32)|id) ^ value bits); block: sum over "
                     "its slices i of mix64(h_i ^ mix64((i<<32)|nnz_i)); sums modulo 2^64; mix64 = SplitMix64 "
                     "output function",
           "semirings": {}}
    for sr, M in (("or_and_bool", H.with_values(None)), ("min_plus_i32", H)):
        t0 = time.time()
        nnz = np.empty(n, np.int64)
        h = np.empty(n, np.uint64)
        for r0 in range(0, n, args.rows_per_call):
            r1 = min(n, r0 + args.rows_per_call)
            nnz[r0:r1], h[r0:r1] = oracle.digest(M, M, sr, select=np.arange(r0, r1))
            print(f"{sr}: rows {r1}/{n} ({time.time() - t0:.0f} s)", flush=True)
        bn, bh = oracle.block_digests(nnz, h, 0, BLOCK)
        rec["semirings"][sr] = {"nnz_C": int(nnz.sum()), "block_nnz": [int(x) for x in bn],
                                "block_hash": [f"{int(x):016x}" for x in bh], "seconds": round(time.time() - t0, 1)}
        with open(out, "w") as f:
            json.dump(rec, f, indent=0)
    print(f"wrote {out}")


if __name__ == "__main__":
    main()
