"""Fill the autotune table for the workload shapes and save it as JSON.

    python -m paper_2110_13042_amd.tune [--out PATH] [--quick]

For every (dtype, shape) below, ``Handle.autotune`` times the candidate plans
(leaf cutoff, Strassen depth cap, split-BF16 leaf tile) on synthetic data of
that shape and keeps the fastest under the shape's half-octave bucket.  The
batch entries cover the bucket grid of the 512-problem workload (m in
[256, 8192], n in [64, 2048]).  Entries are per device architecture; a table
loaded on another architecture is ignored.
"""
from __future__ import annotations

import argparse
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
DEFAULT_OUT = os.path.join(HERE, "tune_table.json")

# (dtype name, m, n): the single-problem workloads
SHAPES = [
    ("f64", 1024, 1024),
    ("f32", 8192, 8192), ("bf16x3", 8192, 8192), ("fp8", 8192, 8192),
    ("f32", 16384, 16384), ("bf16x3", 16384, 16384), ("fp8", 16384, 16384),
    ("f32", 262144, 4096), ("bf16x3", 262144, 4096),
]
DTYPES = {"f64": 0, "f32": 1, "bf16x3": 2, "fp8": 3}


def batch_shapes():
    """One representative (m, n) per half-octave bucket of the batch workload."""
    out = []
    for bm in range(16, 27):
        for bn in range(12, 23):
            out.append((int(round(2 ** (bm / 2))), int(round(2 ** (bn / 2)))))
    return out


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=DEFAULT_OUT)
    ap.add_argument("--quick", action="store_true", help="single-problem shapes only")
    args = ap.parse_args()
    import torch
    sys.path.insert(0, os.path.dirname(HERE))
    from paper_2110_13042_amd import ata
    dev = torch.device("cuda:0")
    h = ata.Handle()
    if os.path.exists(args.out):
        h.tune_load(args.out)
    gen = torch.Generator(device=dev)
    gen.manual_seed(20211025)

    def tune(mode, m, n):
        dt = torch.float64 if mode == "f64" else torch.float32
        A = (torch.rand((m, n), generator=gen, device=dev, dtype=dt) * 2 - 1)
        if m == 262144:                  # ill-scaled columns, as in the tall workload
            A *= 10.0 ** (torch.rand((1, n), generator=gen, device=dev, dtype=dt) * 6 - 3)
        t0 = time.perf_counter()
        best = h.autotune(A, DTYPES[mode])
        print(f"[tune] {mode} {m}x{n}: {best} ({time.perf_counter() - t0:.1f} s)", flush=True)
        del A

    for mode, m, n in SHAPES:
        tune(mode, m, n)
        h.tune_save(args.out)
    if not args.quick:
        for mode in ("f32", "bf16x3"):
            for m, n in batch_shapes():
                tune(mode, m, n)
            h.tune_save(args.out)
    h.close()
    print(f"[tune] wrote {args.out}", flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
