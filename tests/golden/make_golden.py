#!/usr/bin/env python3
"""Writes the oracle's results for the full-size workloads into tests/golden/.

Calls only the oracle (oracle/) on the seeded inputs of
paper_2310_17746_amd/workloads.py; nothing here comes from the HIP path.

Files (whitespace-separated text, '#' comments):
  batch4096_seed0.txt   the 4096 batched ranges (seed 0)
  serve2000_seed1.txt   the 2000 served requests (seed 1); the long count job
                        [2, 10^12 + 1) is pinned by pi(10^12) in pi_values.txt
  window_1e12_1e10.txt  the uint64 list of [10^12, 10^12 + 10^10)

Row kinds:
  C <index> <count>                              every range / request
  L <index> <chunk> <first> <last> <n> <digest>  every listed one, per chunk
A list is cut into chunks of 2^24 elements; <first>/<last> are the chunk's
first and last prime, <digest> the first 32 hex digits of the SHA-256 of the
chunk's little-endian uint64 bytes.  (The window file uses index 0.)

    python tests/golden/make_golden.py [--threads N] [--only batch|serve|window]
"""
from __future__ import annotations

import argparse
import hashlib
import os
import sys
import time
from concurrent.futures import ThreadPoolExecutor

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_2310_17746_amd import workloads  # noqa: E402

CHUNK = 1 << 24
WINDOW = (10 ** 12, 10 ** 12 + 10 ** 10)


def chunk_rows(index: int, v: np.ndarray) -> list[str]:
    """L rows of one list (uint64 array)."""
    v = np.ascontiguousarray(v, dtype="<u8")
    rows = []
    for k, s in enumerate(range(0, len(v), CHUNK)):
        c = v[s:s + CHUNK]
        d = hashlib.sha256(c.tobytes()).hexdigest()[:32]
        rows.append("L %d %d %d %d %d %s" % (index, k, int(c[0]), int(c[-1]), len(c), d))
    return rows


def ranges_file(path, title, lo, hi, mode, threads):
    def one(i):
        a, b = int(lo[i]), int(hi[i])
        if mode[i]:
            v = oracle.primes(a, b, elem_bytes=8, threads=1)
            return ["C %d %d" % (i, len(v))] + chunk_rows(i, v)
        return ["C %d %d" % (i, oracle.count(a, b, threads=1))]

    t0 = time.time()
    # longest ranges first, so that the pool is not left waiting on one
    order = sorted(range(len(lo)), key=lambda i: -(int(hi[i]) - int(lo[i])))
    with ThreadPoolExecutor(threads) as ex:
        res = dict(zip(order, ex.map(one, order)))
    with open(path, "w") as f:
        f.write("# %s\n# written by tests/golden/make_golden.py from the oracle (%.0f s)\n"
                % (title, time.time() - t0))
        for i in range(len(lo)):
            f.write("\n".join(res[i]) + "\n")
    print("wrote %s (%.0f s)" % (path, time.time() - t0), flush=True)


def window_file(path, threads):
    t0 = time.time()
    lo, hi = WINDOW
    v = oracle.primes(lo, hi, elem_bytes=8, threads=threads)
    rows = ["C 0 %d" % len(v)] + chunk_rows(0, v)
    with open(path, "w") as f:
        f.write("# uint64 list of [%d, %d)\n# written by tests/golden/make_golden.py from the oracle (%.0f s)\n"
                % (lo, hi, time.time() - t0))
        f.write("\n".join(rows) + "\n")
    print("wrote %s (%.0f s)" % (path, time.time() - t0), flush=True)


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--threads", type=int, default=oracle.default_threads())
    ap.add_argument("--only", choices=["batch", "serve", "window"], default=None)
    args = ap.parse_args()
    if args.only in (None, "window"):
        window_file(os.path.join(HERE, "window_1e12_1e10.txt"), args.threads)
    if args.only in (None, "batch"):
        lo, hi, mode = workloads.batch_ranges(0)
        ranges_file(os.path.join(HERE, "batch4096_seed0.txt"),
                    "4096 batched ranges, workloads.batch_ranges(0)", lo, hi, mode, args.threads)
    if args.only in (None, "serve"):
        lo, hi, mode, _ = workloads.serving_requests(1)
        ranges_file(os.path.join(HERE, "serve2000_seed1.txt"),
                    "2000 served requests, workloads.serving_requests(1)", lo, hi, mode, args.threads)
    return 0


if __name__ == "__main__":
    sys.exit(main())
