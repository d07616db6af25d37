"""Seeded synthetic workloads (inputs only; no sieve arithmetic here).

The paper's workloads are integer ranges, synthetic by nature; these
generators fix the uneven batched and served range mixes exactly:

* batch_ranges: 4096 ranges, lo log-uniform in [10^6, 10^15], length
  log-uniform in [10^3, 10^8], half count-only and half listed (uint64).
* serving_requests: 2000 requests, lo log-uniform in [10^6, 10^14], length
  log-uniform in [10^4, 10^9], 30% listed (uint64), Poisson arrivals given
  as unit-rate exponential gaps (divide by the arrival rate).

Both use numpy's default_rng (PCG64) with the stated seed, draw in the order
written, and floor the log-uniform values to integers.
"""
from __future__ import annotations

import numpy as np


def batch_ranges(seed: int = 0, n: int = 4096):
    """(lo, hi, mode) as uint64, uint64, uint8 arrays; mode 1 = list."""
    rng = np.random.default_rng(seed)
    lo = np.floor(10 ** rng.uniform(6, 15, n)).astype(np.uint64)
    ln = np.floor(10 ** rng.uniform(3, 8, n)).astype(np.uint64)
    mode = rng.permutation(np.array([0] * (n // 2) + [1] * (n - n // 2), dtype=np.uint8))
    return lo, lo + ln, mode


def serving_requests(seed: int = 1, n: int = 2000):
    """(lo, hi, mode, gaps): gaps are unit-rate exponential inter-arrival times."""
    rng = np.random.default_rng(seed)
    lo = np.floor(10 ** rng.uniform(6, 14, n)).astype(np.uint64)
    ln = np.floor(10 ** rng.uniform(4, 9, n)).astype(np.uint64)
    mode = (rng.random(n) < 0.3).astype(np.uint8)
    gaps = rng.exponential(1.0, n)
    return lo, lo + ln, mode, gaps


# The long count-only job served beside the requests: primes in [2, 10^12].
LONG_JOB = (2, 10 ** 12 + 1)
