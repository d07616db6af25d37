"""Host-side logic of the library, checked on the CPU (no device work).

* The C ABI loads and exports every function include/sieve.h declares.
* Table 1 as evaluated by the library's own wheel code (compiled for the
  host) equals the oracle's definition "first multiple of P >= M in the
  class", and reproduces the paper's worked example (Sec. 3).
* The tile planner covers every wheel value of a range exactly once.
* sieve_list_bound is an upper bound on the oracle's counts.
"""
import math
import os
import random
import re

import pytest

import oracle
from oracle import wheel
from conftest import ROOT, read_golden

pkg = pytest.importorskip("paper_2310_17746_amd")


def _declared_functions():
    names = {}
    inc = os.path.join(ROOT, "include")
    for fn in sorted(os.listdir(inc)):
        if fn.endswith(".h"):
            hdr = re.sub(r"/\*.*?\*/", "", open(os.path.join(inc, fn)).read(), flags=re.S)
            names[fn] = sorted(set(re.findall(r"\b(sieve_[a-z_0-9]+)\s*\(", hdr)))
    return names


def test_library_exports_every_declared_symbol():
    """libsieve.so exports every function of the product headers; the
    mark-counting build exports those and sieve_debug.h's as well."""
    import ctypes
    lib = pkg.load_library()
    dbg = ctypes.CDLL(os.path.join(ROOT, "paper_2310_17746_amd", "libsieve_markcount.so"))
    names = _declared_functions()
    product = [n for fn, ns in names.items() if fn != "sieve_debug.h" for n in ns]
    assert "sieve_count" in product and "sieve_list_batch" in product
    assert names["sieve_debug.h"] == ["sieve_debug_tally"]
    for name in product:
        assert hasattr(lib, name), name
        assert hasattr(dbg, name), name
    assert hasattr(dbg, "sieve_debug_tally") and not hasattr(lib, "sieve_debug_tally")


def test_worked_example_through_library():
    (row,) = read_golden("table1_worked_example.txt")
    P, base, M, Q, q, p, R, idx0, id1, id5, v1, v5 = map(int, row)
    assert pkg.wheel_start(P, base, M) == (id1, id5)


def test_library_table1_equals_oracle_definition():
    rng = random.Random(17)
    primes = oracle.simple_primes(3000).tolist()[2:]  # >= 5
    primes += [65537, 1000003, 31622777, 2147483647, 4294967291]
    n = 0
    for P in primes:
        for _ in range(12):
            base = 6 * rng.randrange(0, 10 ** 13)
            if rng.random() < 0.3:  # segments just below P^2, where M = P^2
                base = max(0, P * P - 6 * rng.randrange(1, 10 ** 6)) // 6 * 6
            M = max(base, rng.choice([base, base + rng.randrange(1, 6 * P + 7), P * P]))
            if M - base >= 2 ** 22:
                M = base + rng.randrange(0, 2 ** 22)
            M = max(M, 1)
            got = pkg.wheel_start(P, base, M)
            want = (wheel.first_multiple_index(P, base, M, 1),
                    wheel.first_multiple_index(P, base, M, 5))
            assert got == want, (P, base, M)
            n += 1
    # exhaustive small corner: every M in a window around P^2 and base
    for P in (5, 7, 11, 13, 17, 19, 23, 29, 31, 37, 41, 43):
        for base in (0, 6, 12000, 6 * 10 ** 15):
            for M in range(max(1, base), base + 8 * P):  # all within 2^22 of base
                assert pkg.wheel_start(P, base, M) == (
                    wheel.first_multiple_index(P, base, M, 1),
                    wheel.first_multiple_index(P, base, M, 5)), (P, base, M)
                n += 1
    assert n > 5000


def test_wheel_start_rejects_bad_input():
    with pytest.raises(pkg.SieveError):
        pkg.wheel_start(9, 0, 10)   # 9 = 3 mod 6 is not a wheel prime
    with pytest.raises(pkg.SieveError):
        pkg.wheel_start(7, 5, 10)   # base not a multiple of 6


@pytest.mark.parametrize("seg", [8192, 65536, 131072, 163840])
def test_plan_covers_every_wheel_value_once(seg):
    rng = random.Random(seg)
    pw = seg // 8
    per_tile = 192 * pw
    cases = [(0, 0), (0, 1), (0, 2), (2, 5), (5, 6), (0, 10 ** 7 + 1), (10 ** 12, 10 ** 12 + 10 ** 10)]
    cases += [(a, a + rng.randrange(0, 4 * per_tile)) for a in
              (rng.randrange(0, 10 ** 15) for _ in range(200))]
    for lo, hi in cases:
        ntiles, base, last = pkg.plan_range(lo, hi, seg)
        assert base % 6 == 0 and base <= lo < base + 6
        # the tiles span [base, base + 192 * words), where words counts A_one words
        words = (ntiles - 1) * pw + last if ntiles else 0
        end = base + 192 * words
        vals_lo = [v for v in range(lo, min(hi, lo + 12)) if v % 6 in (1, 5)]
        vals_hi = [v for v in range(max(lo, hi - 12), hi) if v % 6 in (1, 5)]
        for v in vals_lo + vals_hi:
            assert base <= v < end, (lo, hi, v)
        if ntiles:
            assert 1 <= last <= pw
            assert end - 192 < hi or hi <= base + 1  # no whole word beyond hi
        else:
            assert not [v for v in range(lo, hi) if v % 6 in (1, 5) and v > 1]


def test_list_bound_is_an_upper_bound():
    rng = random.Random(2)
    cases = [(0, 0), (0, 1), (0, 2), (0, 3), (0, 4), (2, 3), (0, 100), (0, 10 ** 6),
             (10 ** 9, 10 ** 9 + 1000)]
    cases += [(a, a + rng.randrange(0, 200000)) for a in (rng.randrange(0, 10 ** 12) for _ in range(60))]
    for lo, hi in cases:
        c = oracle.count(lo, hi)
        b = pkg.list_bound(lo, hi)
        assert b >= c, (lo, hi, b, c)
        if hi - lo > 10 ** 5:
            assert b <= 6 * c + 100  # not vacuous (2y/ln y vs y/ln x)


def test_table1_remainder_edges():
    """The library's remainder of M - 1 by P (invariant reciprocal, 32-bit
    correction below P = 2^31): bases at multiples of P and one off, near
    2^52 and near P^2, all against the oracle's definition."""
    from oracle import brute
    rng = random.Random(23)
    big = [p for p in range(2 ** 30 - 200, 2 ** 30) if brute.is_prime_mr(p)][-3:]
    big += [p for p in range(2 ** 29 - 100, 2 ** 29 + 100) if brute.is_prime_mr(p)][:3]
    small = [5, 7, 67, 1009, 65537, 31622771]
    n = 0
    for P in small + big:
        bases = []
        for top in (2 ** 52, 2 ** 52 - 6 * 1000, 10 ** 15, 6 * 10 ** 12):
            k = top // P
            for mult in (k - 1, k, k + 1):
                for d in (-7, -1, 0, 1, 5, 6):
                    b = (mult * P + d) // 6 * 6
                    if b >= 0:
                        bases.append(b)
        bases += [6 * rng.randrange(0, 2 ** 49) for _ in range(20)]
        for base in bases:
            M = max(base, P * P) if P * P - base < 2 ** 22 else base
            M = max(M, 1)
            got = pkg.wheel_start(P, base, M)
            want = (wheel.first_multiple_index(P, base, M, 1),
                    wheel.first_multiple_index(P, base, M, 5))
            assert got == want, (P, base, M)
            n += 1
    assert n > 1000



def test_first_mismatch_helper():
    from conftest import first_mismatch
    assert first_mismatch([2, 3, 5], [2, 3, 5]) is None
    assert first_mismatch([2, 3, 7, 11], [2, 3, 5, 7])[0] == 2
    assert first_mismatch([2, 3], [2, 3, 5]) == (2, [2, 3], [2, 3, 5])


def test_bench_mark_count_against_brute_force():
    # the roofline's algorithmic LDS work: multiples p*m of every base prime
    # p > 73 from max(p^2, base) to the end of the last plane word, with m
    # coprime to 30 (2 and 3 are off the wheel, 5 is presieved)
    import bench
    rng = random.Random(12)
    for _ in range(60):
        lo = rng.randrange(0, 3 * 10 ** 5)
        hi = lo + rng.randrange(1, 2 * 10 ** 4)
        marks, words = bench.lds_work(lo, hi, 53248)
        base = lo - lo % 6
        end = base + 192 * words
        want = 0
        for p in range(79, math.isqrt(hi - 1) + 1):
            if all(p % q for q in range(2, math.isqrt(p) + 1)):
                for v in range(max(p * p, base), end):
                    if v % p == 0 and math.gcd(v // p, 30) == 1:
                        want += 1
        assert marks == want, (lo, hi)
        assert words == (((hi - base - 1 + 5) // 6) + 31) // 32


def test_bench_refuses_several_gpus():
    # the multi-GPU request is refused before anything touches a device
    import subprocess
    import sys
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""
