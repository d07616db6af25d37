"""Windows beyond the 64-bit calls' domain (Sec. 6: ranges past 2^64 are the
method's next step): sieve_count_wide / sieve_list_wide against the wide
oracle (unsigned 128-bit arithmetic, pinned by deterministic Miller-Rabin),
element by element.

Windows span several tiles with ragged ends, just above 2^64, straddling
2^64, between 2^63 (the end of the 64-bit calls' domain) and 2^64, at the
lowest allowed base 2^40 (where the 64-bit path gives the same list), and
past 2^66, where the base primes reach beyond 2^32 into the 64-bit extension
list.  Edge cases: empty windows, windows with no wheel value, the argument
limits, missing base primes and a short output buffer.
"""
import math
import random

import numpy as np
import pytest

import oracle
from oracle import brute

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
pkg = pytest.importorskip("paper_2310_17746_amd")

T64 = 1 << 64


@pytest.fixture(scope="module")
def sv():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    s = pkg.Sieve(0)
    print("wide: resident base primes below 2^32", flush=True)
    s.base_primes((1 << 32) - 1)
    yield s
    s.close()


def _check_window(sv, lo, hi):
    print("wide: list [%d, %d)" % (lo, hi), flush=True)
    got = sv.list_wide(lo, hi)
    want = oracle.primes_wide(lo, hi)
    g = got.cpu().numpy().view(np.uint64).reshape(-1, 2)
    assert g.shape == want.shape, (lo, hi, g.shape, want.shape)
    if len(want):
        bad = np.nonzero((g != want).any(axis=1))[0]
        assert len(bad) == 0, (lo, hi, int(bad[0]), g[bad[0]], want[bad[0]])
    assert sv.count_wide(lo, hi) == len(want)
    return g


WINDOWS = [
    (T64, T64 + 10 ** 7),                                  # three tiles, ragged last one
    (T64 + 12345, T64 + 12345 + 3 * 10 ** 6 + 7),          # ragged both ends
    (T64 - 4 * 10 ** 6 - 1, T64 + 4 * 10 ** 6 + 3),        # straddles 2^64
    ((1 << 63) + 5, (1 << 63) + 2 * 10 ** 6),              # past the 64-bit calls' end
]


@pytest.mark.parametrize("lo,hi", WINDOWS)
def test_list_wide_matches_oracle(sv, lo, hi):
    _check_window(sv, lo, hi)


def test_wide_at_2_40_equals_64bit_path(sv):
    lo, hi = 1 << 40, (1 << 40) + 5 * 10 ** 6 + 1
    g = _check_window(sv, lo, hi)
    assert np.all(g[:, 1] == 0)
    narrow = sv.list(lo, hi, elem_bytes=8).cpu().numpy().view(np.uint64)
    assert np.array_equal(g[:, 0], narrow)


def test_count_wide_large_window(sv):
    lo, hi = T64 + 10 ** 9, T64 + 10 ** 9 + 10 ** 8
    print("wide: count [%d, %d)" % (lo, hi), flush=True)
    assert sv.count_wide(lo, hi) == oracle.count_wide(lo, hi)


def test_tiny_and_empty_windows(sv):
    base = T64 + 6000
    base -= base % 6
    for a in range(0, 8):
        for b in range(a, 14):
            lo, hi = base + a, base + b
            want = [p for p in range(lo, hi) if brute.is_prime_mr(p)]
            assert sv.count_wide(lo, hi) == len(want), (a, b)
            got = pkg.wide_values(sv.list_wide(lo, hi))
            assert got == want, (a, b)


def test_argument_limits(sv):
    with pytest.raises(pkg.SieveError) as e:
        sv.count_wide((1 << 40) - 1, 1 << 41)
    assert e.value.code == pkg.SIEVE_E_INVAL
    with pytest.raises(pkg.SieveError) as e:
        sv.count_wide(T64, T64 + (1 << 40) + 1)
    assert e.value.code == pkg.SIEVE_E_INVAL
    with pytest.raises(pkg.SieveError) as e:
        sv.count_wide(T64 + 10, T64 + 9)
    assert e.value.code == pkg.SIEVE_E_INVAL
    # base primes end below 2^32 and no extension list: 2^66 needs primes to 2^33
    with pytest.raises(pkg.SieveError) as e:
        sv.count_wide(1 << 66, (1 << 66) + 100)
    assert e.value.code == pkg.SIEVE_E_RANGE
    with pytest.raises(pkg.SieveError) as e:
        sv.base_primes_wide(pkg.WIDE_MAX_BASE + 1)
    assert e.value.code == pkg.SIEVE_E_INVAL


def test_short_output_reports_capacity(sv):
    lo, hi = T64, T64 + 10 ** 5
    n = sv.count_wide(lo, hi)
    out = torch.empty((n - 1, 2), dtype=torch.int64, device="cuda")
    with pytest.raises(pkg.SieveError) as e:
        sv.list_wide(lo, hi, out=out)
    assert e.value.code == pkg.SIEVE_E_CAPACITY
    out = torch.empty((n, 2), dtype=torch.int64, device="cuda")
    assert sv.list_wide(lo, hi, out=out).shape[0] == n


def test_missing_base_primes_is_range_error():
    with pkg.Sieve(0) as s:
        s.base_primes(1 << 20)
        with pytest.raises(pkg.SieveError) as e:
            s.count_wide(T64, T64 + 1000)
        assert e.value.code == pkg.SIEVE_E_RANGE


def test_extension_primes_past_2_66(sv):
    lo, hi = (1 << 66) - 10 ** 6 - 3, (1 << 66) + 10 ** 6
    root = math.isqrt(hi - 1)
    print("wide: extension primes to %d" % root, flush=True)
    n = sv.base_primes_wide(root)
    assert sv.ext_limit == root
    assert n == oracle.count(5, root + 1)  # resident and extension primes >= 5
    g = _check_window(sv, lo, hi)
    _check_window(sv, 3 * T64 + 7, 3 * T64 + 7 + 5 * 10 ** 5)  # high half 3
    # independent spot check: deterministic Miller-Rabin on sampled wheel values
    vals = set(int(h) << 64 | int(l) for l, h in g)
    rng = random.Random(7)
    for _ in range(300):
        v = rng.randrange(lo, hi)
        v += (1 - v % 6) % 6
        if v < hi:
            assert (v in vals) == brute.is_prime_mr(v), v


def test_wide_list_at_bench_size(sv):
    """The bench's wide list, [2^64, 2^64 + 10^9) at the default launch shape:
    sorted, in range, on the wheel; the oracle's list on sampled sub-windows
    and across sampled tile seams; Miller-Rabin on sampled members and
    non-members; the count equals the list length and the sum of the counts
    of ten pieces."""
    lo, hi = T64, T64 + 10 ** 9
    print("wide: bench-size list [%d, %d)" % (lo, hi), flush=True)
    g = sv.list_wide(lo, hi).cpu().numpy().view(np.uint64).reshape(-1, 2)
    assert np.all(g[:, 1] == 1)  # every value in [2^64, 2^65)
    low = g[:, 0]
    assert np.all(low[1:] > low[:-1])
    assert int(low[-1]) < hi - T64 and int(low[0]) >= 0
    r6 = (low + np.uint64(T64 % 6)) % np.uint64(6)
    assert set(np.unique(r6).tolist()) <= {1, 5}
    n = len(low)
    assert sv.count_wide(lo, hi) == n
    step = 10 ** 8
    assert sum(sv.count_wide(lo + k * step, lo + (k + 1) * step) for k in range(10)) == n
    # sub-windows: random offsets, the first and last tile seams and six
    # random ones (tiles of 192 * pw integers)
    pw = sv.params.segment_bytes // 8
    span = 192 * pw
    nseam = (hi - lo) // span
    rng = np.random.default_rng(11)
    offs = [int(x) for x in rng.integers(0, hi - lo - 10 ** 6, 4)]
    offs += [k * span - 50000 for k in [1, nseam] + [int(x) for x in rng.integers(2, nseam, 6)]]
    for o in offs:
        a, b = lo + max(o, 0), min(lo + max(o, 0) + 10 ** 5, hi)
        want = oracle.primes_wide(a, b)
        sel = (low >= np.uint64(a - T64)) & (low < np.uint64(b - T64))
        got = low[sel]
        assert np.array_equal(got, want[:, 0]) and np.all(want[:, 1] == 1), (a, b)
    members = set(int(x) for x in low[rng.integers(0, n, 100)])
    for v in members:
        assert brute.is_prime_mr(T64 + v)
    cand = 0
    while cand < 100:
        v = int(rng.integers(0, hi - lo))
        v += (1 - (T64 + v) % 6) % 6
        if v < hi - lo:
            cand += 1
            k = int(np.searchsorted(low, np.uint64(v)))
            assert (k < n and int(low[k]) == v) == brute.is_prime_mr(T64 + v), v



def test_every_wheel_candidate_by_miller_rabin(sv):
    """Deterministic Miller-Rabin (first twelve prime bases, exact below
    3.18e23) on every wheel candidate of a window just above 2^64, straight
    against the GPU list: a candidate is listed exactly when it is prime."""
    lo, hi = T64 + 10 ** 12 + 1, T64 + 10 ** 12 + 300001
    sv.ensure_base_wide_for(hi)  # isqrt(hi - 1) = 2^32 + 116: the extension list starts here
    assert sv.ext_limit >= 2 ** 32 + 116
    got = set(pkg.wide_values(sv.list_wide(lo, hi)))
    v = lo + (1 - lo % 6) % 6  # first candidate = 1 (mod 6)
    n = 0
    while v < hi:
        for c in (v, v + 4):
            if lo <= c < hi:
                assert (c in got) == brute.is_prime_mr(c), c
                n += 1
        v += 6
    assert n >= 99000 and all(lo <= p < hi and p % 6 in (1, 5) for p in got)


def test_pieces_under_a_small_bucket_budget(sv):
    """With 1 MiB of bucket memory a window runs as many equal pieces, each
    sieved from its own base: the same list and count as one piece, the
    oracle's list, and a short output still reports the full count."""
    lo, hi = T64 + 7, T64 + 2 * 10 ** 7 + 3
    want = oracle.primes_wide(lo, hi)
    one = sv.list_wide(lo, hi).cpu().numpy().view(np.uint64).reshape(-1, 2)
    with pkg.Sieve(0, dict(bucket_mem_mb=1)) as s:
        s.base_primes((1 << 32) - 1)
        print("wide: pieces [%d, %d)" % (lo, hi), flush=True)
        got = s.list_wide(lo, hi).cpu().numpy().view(np.uint64).reshape(-1, 2)
        assert np.array_equal(got, want) and np.array_equal(one, want)
        assert s.count_wide(lo, hi) == len(want)
        out = torch.empty((len(want) // 2, 2), dtype=torch.int64, device="cuda")
        with pytest.raises(pkg.SieveError) as e:
            s.list_wide(lo, hi, out=out)
        assert e.value.code == pkg.SIEVE_E_CAPACITY


def test_values_near_2_127(sv):
    # the 128-bit square root of such bounds needs base primes near 2^63.5
    for lo in (1 << 127, (1 << 128) - 100):
        with pytest.raises(pkg.SieveError) as e:
            sv.count_wide(lo, lo + 10)
        assert e.value.code == pkg.SIEVE_E_RANGE
    with pytest.raises(ValueError):
        pkg.U128.of(1 << 128)


@pytest.fixture(scope="module")
def param_window():
    lo, hi = T64 + 5, T64 + 3 * 10 ** 6 + 11
    return lo, hi, oracle.primes_wide(lo, hi)


@pytest.mark.parametrize("params", [
    dict(segment_bytes=8192, block_threads=256),
    dict(segment_bytes=53248, block_threads=512, wg_per_cu=3),
    dict(presieve_groups=pkg.PRESIEVE_NONE, cofactor_skip=pkg.SKIP_NONE),
    dict(presieve_groups=1, cofactor_skip=pkg.SKIP_ALL, split_hits=8),
    dict(dense_hits=pkg.DENSE_NEVER, split_hits=256),
    dict(segment_bytes=131072, block_threads=1024, bucket_mem_mb=1),
])
def test_wide_under_other_parameters(param_window, params):
    """Tile size, presieve groups, cofactor skip, split and dense items and the
    bucket budget all shape the wide path's work: the list stays the oracle's."""
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    lo, hi, want = param_window
    print("wide params: %s" % params, flush=True)
    with pkg.Sieve(0, params) as s:
        s.base_primes((1 << 32) - 1)
        got = s.list_wide(lo, hi).cpu().numpy().view(np.uint64).reshape(-1, 2)
        assert np.array_equal(got, want), params
        assert s.count_wide(lo, hi) == len(want)
