"""The oracle pinned to things other than itself (CPU only).

Pins: trial division (exhaustive on tiny ranges), deterministic Miller-Rabin
on windows near 10^12 and 10^15, published pi(x) values, the paper's worked
example of Table 1 and its Fig. 2 sequences, invariants of every output
(order, range, residue mod 6, additivity), and the closed-form mark count
against direct enumeration.
"""
import math
import random

import numpy as np
import pytest

import oracle
from oracle import brute, wheel
from conftest import read_golden


# --------------------------------------------------------------------------
# isqrt (step 1 of the oracle)
# --------------------------------------------------------------------------
def test_isqrt_against_math_isqrt():
    rng = random.Random(7)
    vals = list(range(0, 2000))
    for k in range(1, 3100000000, 99991):
        vals += [k * k - 1, k * k, k * k + 1]
    vals += [rng.randrange(0, 1 << 63) for _ in range(2000)]
    vals += [(1 << 63) - 1, 1 << 63, (1 << 64) - 1, 10 ** 15 + 10 ** 8, 10 ** 12 + 10 ** 10 - 1]
    for v in vals:
        assert oracle.isqrt(v) == math.isqrt(v), v


# --------------------------------------------------------------------------
# Trial division, exhaustive on tiny ranges
# --------------------------------------------------------------------------
def test_count_exhaustive_small_ranges():
    N = 400
    isp = [brute.is_prime_td(n) for n in range(N + 1)]
    pref = [0]
    for n in range(N + 1):
        pref.append(pref[-1] + isp[n])
    for lo in range(0, N + 1):
        for hi in range(lo, N + 1):
            assert oracle.count(lo, hi, threads=1) == pref[hi] - pref[lo], (lo, hi)


def test_list_against_trial_division():
    got = oracle.primes(0, 30000, elem_bytes=4)
    assert got.tolist() == brute.primes_td(0, 30000)
    rng = random.Random(11)
    for _ in range(20):
        lo = rng.randrange(0, 3_000_000)
        hi = lo + rng.randrange(0, 3000)
        assert oracle.primes(lo, hi, elem_bytes=8, threads=2).tolist() == brute.primes_td(lo, hi)


def test_window_boundaries():
    # Ranges that straddle the oracle's 2^21-integer windows.
    W = 1 << 21
    for lo, hi in [(W - 50, W + 50), (2 * W - 1, 2 * W + 1), (W, W), (0, W + 1)]:
        got = oracle.primes(lo, hi, elem_bytes=8, threads=3)
        want = [n for n in range(lo, hi) if brute.is_prime_mr(n)]
        assert got.tolist() == want


# --------------------------------------------------------------------------
# Miller-Rabin, and large windows checked with it
# --------------------------------------------------------------------------
def test_miller_rabin_against_trial_division():
    for n in range(0, 50000):
        assert brute.is_prime_mr(n) == brute.is_prime_td(n), n


def test_miller_rabin_known_composites_and_primes():
    # Carmichael numbers and strong pseudoprimes to small bases; each is
    # factored here by trial division so the pin does not rest on memory.
    for n in [561, 1105, 1729, 2465, 2821, 6601, 2047, 3277, 4033, 4681, 8321,
              25326001, 3215031751, 2152302898747, 3474749660383, 341550071728321]:
        f = next(d for d in range(2, math.isqrt(n) + 1) if n % d == 0)
        assert n % f == 0 and 1 < f < n
        assert not brute.is_prime_mr(n), n
    for n in [2 ** 31 - 1, 2 ** 61 - 1, 1000000007, 998244353, 10 ** 12 + 39]:
        assert brute.is_prime_mr(n), n


@pytest.mark.parametrize("lo,length", [(10 ** 12, 200_000), (10 ** 15, 20_000),
                                       (2 ** 32 - 10_000, 20_000)])
def test_large_windows_against_miller_rabin(lo, length):
    hi = lo + length
    got = oracle.primes(lo, hi, elem_bytes=8)
    want = [n for n in range(lo, hi) if brute.is_prime_mr(n)]
    assert got.tolist() == want


# --------------------------------------------------------------------------
# Published values of pi(x)
# --------------------------------------------------------------------------
@pytest.mark.parametrize("x", [10, 100, 1000, 10000, 100000, 10 ** 6, 10 ** 7, 10 ** 8,
                               10 ** 9])
def test_pi_values(pi_table, x):
    assert oracle.count(2, x + 1) == pi_table[x]


@pytest.mark.slow
@pytest.mark.parametrize("x", [2 ** 32, 10 ** 10])
def test_pi_values_slow(pi_table, x):
    assert oracle.count(0, x + 1) == pi_table[x]


def test_simple_sieve(pi_table):
    assert oracle.simple_primes(10000).tolist() == brute.primes_td(0, 10001)
    assert len(oracle.simple_primes(10 ** 6)) == pi_table[10 ** 6]


# --------------------------------------------------------------------------
# Invariants of every output
# --------------------------------------------------------------------------
def test_invariants_and_additivity():
    rng = random.Random(3)
    for _ in range(12):
        a = rng.randrange(0, 10 ** 12)
        c = a + rng.randrange(0, 3_000_000)
        b = rng.randrange(a, c + 1)
        lac = oracle.primes(a, c)
        lab = oracle.primes(a, b)
        lbc = oracle.primes(b, c)
        assert np.array_equal(lac, np.concatenate([lab, lbc]))
        assert len(lac) == oracle.count(a, c) == oracle.count(a, b) + oracle.count(b, c)
        if len(lac):
            assert np.all(np.diff(lac.astype(np.int64)) > 0)
            assert lac[0] >= a and lac[-1] < c
            big = lac[lac > 3]
            assert np.all((big % 6 == 1) | (big % 6 == 5))


def test_u32_and_u64_lists_agree():
    a = oracle.primes(4_000_000_000, 4_000_100_000, elem_bytes=4)
    b = oracle.primes(4_000_000_000, 4_000_100_000, elem_bytes=8)
    assert a.dtype == np.uint32 and b.dtype == np.uint64
    assert np.array_equal(a.astype(np.uint64), b)


def test_invalid_ranges_rejected():
    with pytest.raises(ValueError):
        oracle.count(10, 5)
    with pytest.raises(ValueError):
        oracle.primes(0, 2 ** 32 + 1, elem_bytes=4)
    assert oracle.count(7, 7) == 0


# --------------------------------------------------------------------------
# Fig. 2 and Table 1 (Sec. 2.1, Sec. 3)
# --------------------------------------------------------------------------
def test_fig2_plane_mapping():
    rows = {r[0]: [int(x) for x in r[1:]] for r in read_golden("fig2_planes.txt")}
    assert [wheel.value_of(0, 1, i) for i in range(1, 8)] == rows["A_one"]
    assert [wheel.value_of(0, 5, i) for i in range(0, 7)] == rows["A_five"]
    listed = set(oracle.primes(0, 48).tolist())
    for v in rows["A_one"] + rows["A_five"]:
        assert (v in listed) == (v not in rows["composite"]), v


def test_table1_worked_example():
    (row,) = read_golden("table1_worked_example.txt")
    P, base, M, Q, q, p, R, idx0, id1, id5, v1, v5 = map(int, row)
    assert P * ((M - 1) // P) == Q and Q % 6 == q and P % 6 == p and P // 6 == R
    assert (Q - base) // 6 == idx0
    assert wheel.table1_start(P, base, M) == (id1, id5)
    assert wheel.value_of(base, 1, id1) == v1 and wheel.value_of(base, 5, id5) == v5
    assert v1 % P == 0 and v5 % P == 0


def test_table1_equals_definition():
    primes = [p for p in brute.primes_td(5, 400)] + [1009, 7919, 65537, 104729, 1000003]
    rng = random.Random(5)
    cases = 0
    for P in primes:
        bases = [0, 6, 600, 12000, 6 * 10 ** 6, 6 * rng.randrange(0, 10 ** 12)]
        for base in bases:
            Ms = list(range(base + 1, base + 6 * P + 40, max(1, P // 50)))
            Ms += [base + P * k for k in range(0, 8)]
            Ms += [P * P, P * P + 1, P * P - 1]
            for M in Ms:
                if M < 1:
                    continue
                got = wheel.table1_start(P, base, M)
                want = (wheel.first_multiple_index(P, base, M, 1),
                        wheel.first_multiple_index(P, base, M, 5))
                assert got == want, (P, base, M)
                cases += 1
    assert cases > 20000


def test_mark_count_closed_form():
    rng = random.Random(9)
    for _ in range(3000):
        P = rng.choice(brute.primes_td(5, 200))
        lo = rng.randrange(0, 50000)
        hi = lo + rng.randrange(0, 5000)
        direct = sum(1 for v in range(max(P * P, lo), hi)
                     if v % P == 0 and math.gcd(v // P, 6) == 1)
        assert wheel.mark_count(P, lo, hi) == direct
    # The vectorised sum is the scalar closed form summed.
    for _ in range(200):
        ps = brute.primes_td(5, rng.choice([100, 2000, 20000]))
        lo = rng.randrange(0, 10 ** 7)
        hi = lo + rng.randrange(0, 10 ** 6)
        assert wheel.mark_count_sum(ps, lo, hi) == sum(wheel.mark_count(P, lo, hi) for P in ps)
    # Only values coprime to 6 are ever cleared (Sec. 2.1).
    for P in (5, 7, 11):
        for v in range(P * P, 3000, P):
            if math.gcd(v // P, 6) == 1:
                assert v % 6 in (1, 5)


def test_wide_oracle_matches_64bit_oracle_and_brute_force():
    # the 128-bit arithmetic where the 64-bit oracle also applies
    for lo, hi in [(0, 400), (2 ** 50 - 5000, 2 ** 50 + 10 ** 5), (10 ** 12 - 77, 10 ** 12 + 30011)]:
        got = oracle.primes_wide(lo, hi)
        assert np.all(got[:, 1] == 0)
        assert np.array_equal(got[:, 0], oracle.primes(lo, hi, elem_bytes=8))
        assert oracle.count_wide(lo, hi) == len(got)
    assert [int(x) for x in oracle.primes_wide(0, 60)[:, 0]] == brute.primes_td(0, 60)


def test_wide_oracle_beyond_64_bits_against_miller_rabin():
    # every wheel candidate of a window just above 2^64 (Miller-Rabin with the
    # first twelve prime bases is exact there, far below 3.18e23)
    lo, hi = 2 ** 64 + 1, 2 ** 64 + 3001
    got = oracle.primes_wide(lo, hi)
    vals = [int(a) | (int(b) << 64) for a, b in got]
    assert vals == sorted(set(vals)) and all(lo <= v < hi for v in vals)
    want = [v for v in range(lo, hi) if v % 6 in (1, 5) and brute.is_prime_mr(v)]
    assert vals == want
    assert len(vals) > 50
