"""Calibration run for rocprofv3's HBM byte counters.

A plain elementwise kernel of known size (float32 negation: reads N bytes,
writes N bytes, no reuse) is launched a few times.  Profiled with
``rocprofv3 --pmc FETCH_SIZE`` and, in a separate run, ``--pmc WRITE_SIZE``,
its per-dispatch counter values divided by N give the factors by which the
same counters of the SpGEMM kernels are scaled to bytes.

    python3 -m paper_2106_14402_amd.calib --mib 1024 --reps 3
"""
import argparse
import json

import torch


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--mib", type=int, default=1024, help="buffer size in MiB")
    ap.add_argument("--reps", type=int, default=3)
    a = ap.parse_args()
    n = (a.mib << 20) // 4
    x = torch.ones(n, dtype=torch.float32, device="cuda")
    y = torch.empty_like(x)
    torch.cuda.synchronize()
    for _ in range(a.reps):
        torch.neg(x, out=y)
    torch.cuda.synchronize()
    print(json.dumps({"kernel": "neg (float32 elementwise)", "bytes_read": 4 * n, "bytes_written": 4 * n,
                      "reps": a.reps}), flush=True)


if __name__ == "__main__":
    main()
