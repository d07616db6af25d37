"""Marking completeness, through the mark-counting build of the library
(libsieve_markcount.so, include/sieve_debug.h).

Over a range [lo, hi) the tiles cover the wheel values of [B, E), with
B = lo - lo mod 6 and E = B + 192 * ceil(n / 32) for n = ceil((hi - B - 1) / 6)
indices per plane.  Every base prime P above the presieved ones (5..73) with
P * P < hi must visit exactly the multiples m * P with gcd(m, 6) = 1 and
max(P * P, B) <= m * P < E (Sec. 1.1: marking starts at the square;
Sec. 2.1: the arrays hold only values coprime to 6), whichever path marks it:
the per-tile loops (fixed-mask, split or plain items, carried registers,
fresh starts), the parts of a split tile, or the bucket sieve.  The kernels'
tally of visited hits must equal that closed form (oracle.wheel), every
visited hit is either ORed or skipped as a multiple of 5, no run starts on a
value that is not a multiple of its prime at or past the square, and with the
cofactor skip off nothing is skipped.
"""
import ctypes
import math
import os

import numpy as np
import pytest

import oracle
from oracle import wheel

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
pkg = pytest.importorskip("paper_2310_17746_amd")

LIB = os.path.join(os.path.dirname(pkg.__file__), "libsieve_markcount.so")
PRESIEVED_MAX = 73  # the default presieve groups cover the primes 5..73


@pytest.fixture(scope="module")
def dbg():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    lib = ctypes.CDLL(LIB)
    p = ctypes.c_void_p
    u64 = ctypes.c_uint64
    lib.sieve_create.argtypes = [ctypes.POINTER(p), ctypes.c_int, ctypes.POINTER(pkg.Params)]
    lib.sieve_destroy.argtypes = [p]
    lib.sieve_base_primes.argtypes = [p, u64, ctypes.POINTER(u64)]
    lib.sieve_count.argtypes = [p, u64, u64, ctypes.POINTER(u64)]
    lib.sieve_debug_tally.argtypes = [p, ctypes.POINTER(u64), ctypes.c_int]
    return lib


def _expected_hits(lo, hi):
    base = lo - lo % 6
    if hi <= base + 1:
        return 0
    n1 = (hi - base - 1 + 5) // 6
    end = base + 192 * ((n1 + 31) // 32)
    primes = oracle.simple_primes(math.isqrt(hi - 1)).astype(np.int64)
    return wheel.mark_count_sum(primes[primes > PRESIEVED_MAX], base, end)


RANGES = [(10 ** 6, 10 ** 6 + 3 * 10 ** 7), (2, 10 ** 9 + 1), (10 ** 12, 10 ** 12 + 10 ** 8),
          (10 ** 13 + 7, 10 ** 13 + 4 * 10 ** 8 + 3), (10 ** 15, 10 ** 15 + 10 ** 6),
          # last tile of 2306 words: a fixed-mask lane of 461 (32 lanes) has
          # step floor(plane bytes / 5) and a sixth hit in the last word
          (49944454, 87742652)]


@pytest.mark.parametrize("params", [
    {},                                                          # default shape, items + registers
    dict(segment_bytes=53248, block_threads=512, wg_per_cu=3),  # 80-VGPR variant, fresh starts
    dict(strip_tiles=1),                                         # no carried state
    dict(cofactor_skip=pkg.SKIP_NONE),                           # nothing skipped
    dict(cofactor_skip=pkg.SKIP_ALL, dense_hits=pkg.DENSE_NEVER),
    dict(segment_bytes=16384, bucket_threshold=70000),           # most primes through buckets
])
def test_marks_equal_closed_form(dbg, params):
    q = pkg.Params()
    for k, v in params.items():
        setattr(q, k, v)
    h = ctypes.c_void_p()
    assert dbg.sieve_create(ctypes.byref(h), 0, ctypes.byref(q)) == 0
    try:
        n = ctypes.c_uint64()
        assert dbg.sieve_base_primes(h, math.isqrt(max(b for _, b in RANGES)) + 1, ctypes.byref(n)) == 0
        t = (ctypes.c_uint64 * 4)()
        assert dbg.sieve_debug_tally(h, t, 1) == 0
        for lo, hi in RANGES:
            print("marks: %s [%d, %d)" % (params, lo, hi), flush=True)
            c = ctypes.c_uint64()
            assert dbg.sieve_count(h, lo, hi, ctypes.byref(c)) == 0
            assert dbg.sieve_debug_tally(h, t, 1) == 0
            hits, issued, skipped, bad = (int(x) for x in t)
            want = _expected_hits(lo, hi)
            assert bad == 0, (lo, hi, bad)
            assert hits == want, (lo, hi, hits, want)
            assert issued + skipped == hits, (lo, hi, issued, skipped, hits)
            if params.get("cofactor_skip") == pkg.SKIP_NONE:
                assert skipped == 0
            if lo >= 10 ** 12:
                assert c.value == oracle.count(lo, hi), (lo, hi)
    finally:
        dbg.sieve_destroy(h)
