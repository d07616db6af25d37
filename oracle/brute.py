"""Brute-force primality checks -- TEST INFRASTRUCTURE ONLY (see oracle/__init__).

* ``is_prime_td`` / ``primes_td``: trial division, the most literal definition
  of primality; only for small inputs.
* ``is_prime_mr``: deterministic Miller-Rabin with the first twelve primes as
  witnesses.  Sorenson and Webster (Math. Comp. 86, 2017; arXiv 2015) show the
  smallest strong pseudoprime to all of them is psi_12 ~ 3.18e23, so the test
  is exact for every n below that, which covers all 64-bit n.
"""
from __future__ import annotations

_MR_BASES = (2, 3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37)


def is_prime_td(n: int) -> bool:
    """Trial division by every d with d*d <= n."""
    if n < 2:
        return False
    d = 2
    while d * d <= n:
        if n % d == 0:
            return False
        d += 1
    return True


def primes_td(lo: int, hi: int) -> list[int]:
    """Primes of [lo, hi) by trial division (small ranges only)."""
    return [n for n in range(lo, hi) if is_prime_td(n)]


def is_prime_mr(n: int) -> bool:
    """Deterministic Miller-Rabin for n < 3.18e23 (first twelve prime bases)."""
    if n < 2:
        return False
    for p in _MR_BASES:
        if n % p == 0:
            return n == p
    d, s = n - 1, 0
    while d % 2 == 0:
        d //= 2
        s += 1
    for a in _MR_BASES:
        x = pow(a, d, n)
        if x == 1 or x == n - 1:
            continue
        for _ in range(s - 1):
            x = x * x % n
            if x == n - 1:
                break
        else:
            return False
    return True
