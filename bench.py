#!/usr/bin/env python3
"""Benchmark: sieved integers/s counting the primes of [2, 10^11] on one MI355X.

One step = one full pass of the sieve over the workload: a sieve_count call
on [2, 10^11 + 1) (tiling, presieve, Table 1 starts, LDS marking, edge masks,
popcount, per-range total), with the base primes <= isqrt(10^11) already
resident in HBM.  Prints one JSON line.

The roofline entry is for the dominant kernel (k_sieve): its algorithmic LDS
traffic (4 bytes per mark, read-modify-write of one 32-bit word, plus 8 bytes
written per plane-word pair at init and 8 bytes read back by the popcount)
over its average duration, measured with HIP events on the stream it runs
on, against the nominal LDS bandwidth of the chip (128 B/clk/CU * 256 CUs *
2.4 GHz).  The mark count is exact: for every base prime p > 61 the number of
m coprime to 6 with max(p^2, tile base) <= m*p < tile-span end.

The CPU baseline is the oracle (plain byte-per-integer segmented sieve, all
host threads) timed on a bounded slice of the same workload.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PI_1E11 = 4118054813            # pi(10^11), standard published value
LDS_PEAK_GBS = 128 * 256 * 2.4  # nominal LDS bandwidth, GB/s (B/clk/CU * CUs * GHz)


def small_primes(limit: int) -> np.ndarray:
    a = np.ones(limit + 1, dtype=bool)
    a[:2] = False
    for i in range(2, math.isqrt(limit) + 1):
        if a[i]:
            a[i * i::i] = False
    return np.nonzero(a)[0].astype(np.int64)


def coprime6_upto(n: np.ndarray) -> np.ndarray:
    """#{1 <= m <= n : gcd(m, 6) = 1}, elementwise, n >= 0."""
    q, s = np.divmod(n, 6)
    return 2 * q + (s >= 1) + (s >= 5)


def lds_work(lo: int, hi: int, segment_bytes: int) -> tuple[int, int]:
    """(marks, plane words) the sieve kernel performs on [lo, hi)."""
    pw = segment_bytes // 8
    base = lo - lo % 6
    n1 = (hi - base - 1 + 5) // 6
    words = (n1 + 31) // 32
    end = base + 192 * words
    p = small_primes(math.isqrt(hi - 1))
    p = p[p > 61]                                  # 5..61 are presieved by patterns
    ntiles = (words + pw - 1) // pw
    tile_span = 192 * pw
    marks = 0
    # per tile the start is max(p^2, tile base); sum over tiles = over the span
    # with the p^2 clamp, since tiles are contiguous
    start = np.maximum(p * p, base)
    m_lo = -(-start // p)
    m_hi = (end - 1) // p
    ok = m_hi >= m_lo
    marks = int(np.sum(np.where(ok, coprime6_upto(m_hi) - coprime6_upto(m_lo - 1), 0)))
    del ntiles, tile_span
    return marks, int(words)


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--hi", type=int, default=10 ** 11 + 1)
    ap.add_argument("--segment-bytes", type=int, default=0)
    ap.add_argument("--block-threads", type=int, default=0)
    ap.add_argument("--wg-per-cu", type=int, default=0)
    ap.add_argument("--split-hits", type=int, default=0)
    ap.add_argument("--presieve-groups", type=int, default=0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample", type=int, default=10 ** 11,
                    help="integers of the oracle's timed slice (the top of the range)")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(see the sharding design); run with --gpus 1", file=sys.stderr)
        return 2

    import torch
    import paper_2310_17746_amd as pkg

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        return 2
    lo, hi = 2, args.hi
    params = {k: v for k, v in dict(segment_bytes=args.segment_bytes, block_threads=args.block_threads,
                                     wg_per_cu=args.wg_per_cu, split_hits=args.split_hits,
                                     presieve_groups=args.presieve_groups).items() if v}
    s = pkg.Sieve(0, params)
    s.ensure_base_for(hi)                     # base primes resident before timing
    prm = s.params.as_dict()
    print("bench: count [%d, %d) params %s" % (lo, hi, prm), file=sys.stderr, flush=True)

    for _ in range(args.warmup):
        c = s.count(lo, hi)
    torch.cuda.synchronize()
    s.set_timing(True)
    t0 = time.perf_counter()
    for _ in range(args.steps):
        c = s.count(lo, hi)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    sieve_ms, post_ms, jobs = s.timing()
    s.set_timing(False)
    dt = t1 - t0
    ints = hi - lo
    value = ints * args.steps / dt
    count_ok = (c == PI_1E11) if hi == 10 ** 11 + 1 else None

    marks, words = lds_work(lo, hi, prm["segment_bytes"])
    lds_bytes = 4 * marks + 16 * words
    k_ms = sieve_ms / max(jobs, 1)
    achieved = lds_bytes / (k_ms * 1e-3) / 1e9
    roof = {"bound": "alu", "resource": "LDS read-modify-write (32-bit words)",
            "achieved": round(achieved, 1), "peak": round(LDS_PEAK_GBS, 1), "unit": "GB/s",
            "frac": round(achieved / LDS_PEAK_GBS, 4), "traffic": None,
            "kernel": "k_sieve", "kernel_ms": round(k_ms, 4), "marks": marks,
            "algorithmic_bytes": lds_bytes}

    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        th = oracle.default_threads()
        a = max(lo, hi - args.cpu_sample)
        t2 = time.perf_counter()
        oc = oracle.count(a, hi, threads=th)
        t3 = time.perf_counter()
        cpu = {"value": round((hi - a) / (t3 - t2), 1), "unit": "ints/s", "cores": th, "kind": "oracle",
               "sample": "oracle count of [%d, %d) (%d integers, the top of the workload): %d primes in %.2f s"
                         % (a, hi, hi - a, oc, t3 - t2)}

    line = {
        "metric": "sieved integers/s at pi(1e11) count",
        "value": round(value, 1),
        "unit": "ints/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(dt / args.steps * 1e3, 4),
        "higher_is_better": True,
        "scaling": "strong",
        "vs_baseline": None,
        "dtype": "u32",
        "data": "synthetic",
        "config": {"workload": "count the primes in [2, 10^11] (half-open [2, 10^11 + 1))",
                   "lo": lo, "hi": hi, "base_prime_limit": math.isqrt(hi - 1), **prm},
        "count": int(c),
        "count_ok": count_ok,
        "roofline": roof,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)
    s.close()
    return 0 if count_ok is not False else 1


if __name__ == "__main__":
    sys.exit(main())
