"""Wheel index mapping and Table 1 -- TEST INFRASTRUCTURE ONLY (see oracle/__init__).

Index mapping (Sec. 2.1, Fig. 2; the worked example of Sec. 3):
    a chunk with base value B (a multiple of 6) holds two arrays, A_one and
    A_five; entry i of A_r stands for the value B + 6*i + r, r in {1, 5}.

Table 1 (Sec. 3): for a prime P, a chunk base B and a starting value M, the
first entry to clear in each array.  The paper's steps:
    Q  = the greatest multiple of P below M (strictly below; see the readings
         in the design notes: the worked example's 14,391 is the greatest
         multiple of 13 below 14,400),
    q  = Q mod 6,  p = P mod 6 (1 or 5),  R = floor(P / 6),
    idx0 = the index of Q relative to the chunk base, floor((Q - B) / 6),
    then id_1 and id_5 are idx0 plus the Table 1 entry for (p, q).

``table1_start`` follows those steps with the table as printed;
``first_multiple_index`` is the plain definition it must equal ("the index of
the first multiple of P that is >= M and lies in array A_r"), found by walking
up from M.
"""
from __future__ import annotations

# Table 1 as printed, per (p, q): ((a1, b1), (a5, b5)) meaning
# id_1 += a1*R + b1 and id_5 += a5*R + b5.  Entries written "k*(R+1)-1" in the
# paper are expanded to (k, k-1) and "k*(R+1)" to (k, k).
TABLE1 = {
    (1, 0): ((1, 0), (5, 0)),
    (1, 1): ((6, 1), (4, 0)),
    (1, 2): ((5, 1), (3, 0)),
    (1, 3): ((4, 1), (2, 0)),
    (1, 4): ((3, 1), (1, 0)),
    (1, 5): ((2, 1), (6, 1)),
    (5, 0): ((5, 4), (1, 0)),
    (5, 1): ((6, 5), (2, 1)),
    (5, 2): ((1, 1), (3, 2)),
    (5, 3): ((2, 2), (4, 3)),
    (5, 4): ((3, 3), (5, 4)),
    (5, 5): ((4, 4), (6, 5)),
}


def value_of(base: int, r: int, i: int) -> int:
    """Value held by entry i of array A_r in a chunk with base value ``base``."""
    assert base % 6 == 0 and r in (1, 5)
    return base + 6 * i + r


def table1_start(P: int, base: int, M: int) -> tuple[int, int]:
    """(id_1, id_5) for prime P >= 5 by the steps of Sec. 3 and Table 1."""
    assert P >= 5 and P % 6 in (1, 5) and base % 6 == 0 and M >= 1
    Q = P * ((M - 1) // P)          # greatest multiple of P strictly below M
    q = Q % 6
    p = P % 6
    R = P // 6
    idx0 = (Q - base) // 6          # floor, may be negative
    (a1, b1), (a5, b5) = TABLE1[(p, q)]
    return idx0 + a1 * R + b1, idx0 + a5 * R + b5


def first_multiple_index(P: int, base: int, M: int, r: int) -> int:
    """Index in A_r of the first multiple of P that is >= M and = r (mod 6)."""
    assert base % 6 == 0 and r in (1, 5)
    v = P * (-(-M // P))            # first multiple of P >= M
    while v % 6 != r:
        v += P
    return (v - base - r) // 6


def count_coprime6(n: int) -> int:
    """#{1 <= m <= n : gcd(m, 6) = 1} for n >= 0."""
    if n <= 0:
        return 0
    q, s = divmod(n, 6)
    return 2 * q + (1 if s >= 1 else 0) + (1 if s >= 5 else 0)


def mark_count(P: int, lo: int, hi: int) -> int:
    """Marks prime P makes on the wheel arrays over [lo, hi).

    The wheel holds only values coprime to 6, so P clears exactly the values
    m*P with gcd(m, 6) = 1 and max(P*P, lo) <= m*P < hi.  Closed form via
    count_coprime6 on the cofactor interval.
    """
    start = max(P * P, lo)
    if start >= hi:
        return 0
    m_lo = -(-start // P)           # ceil
    m_hi = (hi - 1) // P            # last cofactor with m*P < hi
    if m_hi < m_lo:
        return 0
    return count_coprime6(m_hi) - count_coprime6(m_lo - 1)


def mark_count_sum(primes, lo: int, hi: int) -> int:
    """Sum of mark_count(P, lo, hi) over an array of primes (numpy, int64).

    The same closed form, evaluated for every prime at once: cofactors m in
    [ceil(max(P*P, lo) / P), floor((hi - 1) / P)] counted by count_coprime6.
    Needs P*P and hi below 2^63.
    """
    import numpy as np

    P = np.asarray(primes, dtype=np.int64)
    if P.size == 0 or hi <= lo:
        return 0
    assert int(P.max()) < 3037000499 and hi < 2 ** 63
    start = np.maximum(P * P, np.int64(lo))
    m_lo = -(-start // P)
    m_hi = (np.int64(hi) - 1) // P

    def c6(n):
        n = np.maximum(n, 0)
        q, s = np.divmod(n, 6)
        return 2 * q + (s >= 1) + (s >= 5)

    ok = (start < hi) & (m_hi >= m_lo)
    return int(np.sum(np.where(ok, c6(m_hi) - c6(m_lo - 1), 0)))
