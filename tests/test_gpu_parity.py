"""GPU parity of the HIP sieve against the oracle (bit-exact, tolerance 0).

Every test goes through the C ABI (libsieve.so via the ctypes binding) and
compares with the oracle computed on the same ranges.  Sizes span many tiles
with ragged tails; full-size configurations are checked by count against
published pi(x) values and by list against the oracle.
"""
import math
import random

import numpy as np
import pytest

import oracle
from oracle import brute
from conftest import assert_same_primes, read_golden

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
pkg = pytest.importorskip("paper_2310_17746_amd")


def _u(t, elem_bytes):
    a = t.cpu().numpy()
    return a.view(np.uint32 if elem_bytes == 4 else np.uint64)


@pytest.fixture(scope="module")
def sv():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    s = pkg.Sieve(0)
    s.base_primes(1 << 20)
    yield s
    s.close()


@pytest.fixture(scope="module")
def pi_tab():
    return {int(x): int(v) for x, v in read_golden("pi_values.txt")}


def test_count_tiny_ranges_exhaustive(sv):
    N = 300
    isp = [brute.is_prime_td(n) for n in range(N + 1)]
    pref = np.concatenate([[0], np.cumsum(isp)])
    lo, hi = [], []
    for a in range(N + 1):
        for b in range(a, N + 1):
            lo.append(a)
            hi.append(b)
    got = sv.count_batch(lo, hi).astype(np.int64)
    want = (pref[np.array(hi)] - pref[np.array(lo)]).astype(np.int64)
    bad = np.nonzero(got != want)[0]
    assert len(bad) == 0, [(lo[i], hi[i], int(got[i]), int(want[i])) for i in bad[:10]]
    for a, b in [(0, 0), (0, 2), (0, 3), (0, 4), (2, 3), (3, 4), (4, 5), (5, 6), (1, 2), (0, 8)]:
        assert sv.count(a, b) == int(pref[b] - pref[a]), (a, b)


@pytest.mark.parametrize("lo,hi", [(0, 1_000_000), (0, 100), (1, 7), (5, 6), (24, 50),
                                   (999_983, 2_000_003), (12_000, 18_000)])
def test_list_small_u32(sv, lo, hi):
    got = _u(sv.list(lo, hi, elem_bytes=4), 4)
    want = oracle.primes(lo, hi, elem_bytes=4)
    assert_same_primes(got, want)


def test_list_random_windows_ragged(sv):
    rng = random.Random(1234)
    seg = sv.params.segment_bytes
    tile_vals = 24 * seg
    for _ in range(25):
        lo = rng.randrange(0, 10 ** 12)
        n = rng.choice([0, 1, 7, 191, 192, 193, 12345, tile_vals - 1, tile_vals, tile_vals + 1,
                        3 * tile_vals + rng.randrange(tile_vals)])
        hi = lo + n
        sv.ensure_base_for(hi)
        got = _u(sv.list(lo, hi, elem_bytes=8), 8)
        want = oracle.primes(lo, hi, elem_bytes=8)
        assert_same_primes(got, want, (lo, hi))
        assert sv.count(lo, hi) == len(want), (lo, hi)


def test_full_list_to_1e7(sv, pi_tab):
    lo, hi = 2, 10 ** 7 + 1
    assert sv.count(lo, hi) == pi_tab[10 ** 7]
    got = _u(sv.list(lo, hi, elem_bytes=4), 4)
    want = oracle.primes(lo, hi, elem_bytes=4)
    assert len(got) == pi_tab[10 ** 7]
    assert_same_primes(got, want)


def test_full_list_to_1e9(sv, pi_tab):
    lo, hi = 2, 10 ** 9 + 1
    sv.ensure_base_for(hi)
    assert sv.count(lo, hi) == pi_tab[10 ** 9]
    got = _u(sv.list(lo, hi, elem_bytes=4), 4)
    want = oracle.primes(lo, hi, elem_bytes=4)
    assert len(got) == pi_tab[10 ** 9]
    assert_same_primes(got, want)


def test_pi_1e10_and_1e11_counts(sv, pi_tab):
    sv.ensure_base_for(10 ** 11 + 1)
    assert sv.count(2, 10 ** 10 + 1) == pi_tab[10 ** 10]
    assert sv.count(0, 2 ** 32 + 1) == pi_tab[2 ** 32]
    assert sv.count(2, 10 ** 11 + 1) == pi_tab[10 ** 11]


def test_pi_1e12_count(sv, pi_tab):
    # base primes to 10^6; the bucket sieve takes the primes above four plane lengths
    sv.ensure_base_for(10 ** 12 + 1)
    assert sv.count(2, 10 ** 12 + 1) == pi_tab[10 ** 12]


def test_large_windows_vs_oracle(sv):
    for lo, n in [(10 ** 12, 3 * 10 ** 7), (10 ** 15 - 10 ** 7, 2 * 10 ** 7), (2 ** 50, 10 ** 6)]:
        hi = lo + n
        sv.ensure_base_for(hi)
        got = _u(sv.list(lo, hi, elem_bytes=8), 8)
        want = oracle.primes(lo, hi, elem_bytes=8)
        assert_same_primes(got, want, lo)
        # sampled Miller-Rabin on a few hundred listed values
        for v in got[:: max(1, len(got) // 200)].tolist():
            assert brute.is_prime_mr(int(v))


def test_count_batch_uneven(sv):
    rng = np.random.default_rng(7)
    n = 300
    lo = np.floor(10 ** rng.uniform(0, 13, n)).astype(np.uint64)
    ln = np.floor(10 ** rng.uniform(0, 6.5, n)).astype(np.uint64)
    hi = lo + ln
    sv.ensure_base_for(int(hi.max()))
    got = sv.count_batch(lo, hi)
    want = np.array([oracle.count(int(a), int(b), threads=4) for a, b in zip(lo, hi)], dtype=np.uint64)
    assert_same_primes(got, want)
    # the same ranges alone give the same counts
    for i in range(0, n, 37):
        assert sv.count(int(lo[i]), int(hi[i])) == int(want[i])


def test_list_batch_mixed_and_capacity(sv):
    rng = np.random.default_rng(11)
    n = 64
    lo = np.floor(10 ** rng.uniform(3, 12, n)).astype(np.uint64)
    hi = lo + np.floor(10 ** rng.uniform(0, 6, n)).astype(np.uint64)
    mode = (np.arange(n) % 2).astype(np.uint8)
    sv.ensure_base_for(int(hi.max()))
    want = [oracle.primes(int(a), int(b), elem_bytes=8) for a, b in zip(lo, hi)]
    cap = np.array([pkg.list_bound(int(a), int(b)) for a, b in zip(lo, hi)], dtype=np.uint64)
    cap[5] = max(len(want[5]) - 1, 0) if len(want[5]) else 0   # too small for range 5 (a list range)
    off = np.concatenate([[0], np.cumsum(cap)[:-1]]).astype(np.uint64)
    out = torch.zeros(int(cap.sum()) + 1, dtype=torch.int64, device="cuda")
    counts, status = sv.list_batch(lo, hi, mode, out, off, cap, elem_bytes=8)
    host = _u(out, 8)
    for i in range(n):
        assert int(counts[i]) == len(want[i]), i
        if mode[i] and i == 5 and len(want[5]) > 0:
            assert status[i] == pkg.SIEVE_E_CAPACITY
            continue
        assert status[i] == 0, i
        if mode[i]:
            o = int(off[i])
            assert np.array_equal(host[o:o + len(want[i])], want[i]), i


def test_batch_visit_order_mixed(sv):
    """Tiles are taken in a host-set visit order (most Table 1 starts per tile
    first): empty ranges with large bounds sort first and share their
    successor's visit position; costly single-tile ranges near 10^15 come
    before long low ranges.  Results must not depend on that order."""
    E = 10 ** 15
    spec = [(E, E), (E + 7, E + 7), (5, 5), (E, E + 1), (E + 1, E + 60000),
            (E + 3 * 10 ** 7, E + 3 * 10 ** 7 + 150000), (E // 4, E // 4 + 90000),
            (10 ** 14 + 11, 10 ** 14 + 200011), (10 ** 9, 10 ** 9 + 5 * 10 ** 6),
            (2, 4 * 10 ** 6 + 3), (10 ** 12, 10 ** 12 + 3 * 10 ** 6 + 1), (17, 18), (10 ** 11, 10 ** 11)]
    random.Random(5).shuffle(spec)
    lo = np.array([a for a, _ in spec], dtype=np.uint64)
    hi = np.array([b for _, b in spec], dtype=np.uint64)
    n = len(spec)
    mode = (np.arange(n) % 2).astype(np.uint8)
    sv.ensure_base_for(int(hi.max()))
    want = [oracle.primes(int(a), int(b), elem_bytes=8, threads=4) for a, b in spec]
    assert np.array_equal(sv.count_batch(lo, hi), np.array([len(w) for w in want], dtype=np.uint64))
    cap = np.array([pkg.list_bound(int(a), int(b)) for a, b in spec], dtype=np.uint64)
    off = np.concatenate([[0], np.cumsum(cap)[:-1]]).astype(np.uint64)
    out = torch.zeros(int(cap.sum()) + 1, dtype=torch.int64, device="cuda")
    counts, status = sv.list_batch(lo, hi, mode, out, off, cap, elem_bytes=8)
    host = _u(out, 8)
    for i in range(n):
        assert int(counts[i]) == len(want[i]) and status[i] == 0, spec[i]
        if mode[i]:
            o = int(off[i])
            assert np.array_equal(host[o:o + len(want[i])], want[i]), spec[i]


@pytest.mark.parametrize("lo,hi,params", [
    (10 ** 14 + 3, 10 ** 14 + 400003, {}),                                  # one tile, 664k primes
    (10 ** 15 - 999, 10 ** 15 + 1001, {}),                                  # a few words, 1.9M primes
    (10 ** 14 + 1, 10 ** 14 + 3 * 10 ** 6 + 7, dict(bucket_threshold=pkg.BUCKET_NEVER)),  # 3 tiles
])
def test_split_tiles_small_jobs(lo, hi, params):
    """A small job whose tiles start far more primes than a workgroup's share
    splits them into parts on several workgroups that meet in a global copy
    of the planes; count and list must not notice."""
    with pkg.Sieve(0, params) as s:
        s.ensure_base_for(hi)
        want = oracle.primes(lo, hi, elem_bytes=8, threads=4)
        assert s.count(lo, hi) == len(want)
        got = _u(s.list(lo, hi, elem_bytes=8), 8)
        assert_same_primes(got, want)
        # inside a job whose share per workgroup is larger (pi(10^11): about
        # 2.8M starts per workgroup) the range is not split; counts agree
        los = np.array([lo, 2, lo], dtype=np.uint64)
        his = np.array([hi, 10 ** 11 + 1, hi], dtype=np.uint64)
        c = s.count_batch(los, his)
        assert int(c[0]) == len(want) and int(c[2]) == len(want) and int(c[1]) == 4118054813


def test_random_batch_to_1e15():
    """Seeded uneven batch across nine decades: bucket ranges, split and
    unsplit single tiles and long low ranges in one job, in the host's visit
    order; counts and (for every other range) uint64 lists against the oracle."""
    rng = np.random.default_rng(23)
    n = 128
    lo = np.floor(10 ** rng.uniform(6, 15, n)).astype(np.uint64)
    hi = lo + np.floor(10 ** rng.uniform(3, 7, n)).astype(np.uint64)
    mode = (np.arange(n) % 2).astype(np.uint8)
    with pkg.Sieve(0) as s:
        s.ensure_base_for(int(hi.max()))
        want = [oracle.primes(int(a), int(b), elem_bytes=8, threads=4) for a, b in zip(lo, hi)]
        assert np.array_equal(s.count_batch(lo, hi), np.array([len(w) for w in want], dtype=np.uint64))
        cap = np.array([pkg.list_bound(int(a), int(b)) if m else 0 for a, b, m in zip(lo, hi, mode)],
                       dtype=np.uint64)
        off = np.concatenate([[0], np.cumsum(cap)[:-1]]).astype(np.uint64)
        out = torch.zeros(int(cap.sum()) + 1, dtype=torch.int64, device="cuda")
        counts, status = s.list_batch(lo, hi, mode, out, off, cap, elem_bytes=8)
        host = _u(out, 8)
        for i in range(n):
            assert int(counts[i]) == len(want[i]) and status[i] == 0, (int(lo[i]), int(hi[i]))
            if mode[i]:
                o = int(off[i])
                assert np.array_equal(host[o:o + len(want[i])], want[i]), (int(lo[i]), int(hi[i]))


def test_capacity_error_reports_count(sv):
    n_true = oracle.count(10 ** 6, 2 * 10 ** 6)
    out = torch.empty(10, dtype=torch.int64, device="cuda")
    with pytest.raises(pkg.SieveError) as ei:
        sv.list(10 ** 6, 2 * 10 ** 6, out=out, elem_bytes=8)
    assert ei.value.code == pkg.SIEVE_E_CAPACITY
    assert sv.count_list(10 ** 6, 2 * 10 ** 6) == n_true


def test_error_paths(sv):
    with pytest.raises(pkg.SieveError) as ei:
        sv.count(10, 5)
    assert ei.value.code == pkg.SIEVE_E_INVAL
    with pytest.raises(pkg.SieveError) as ei:
        sv.count(0, 2 ** 63 + 1)
    assert ei.value.code == pkg.SIEVE_E_INVAL
    lim = sv.base_limit
    with pytest.raises(pkg.SieveError) as ei:
        sv.count(0, (lim + 1) ** 2 + 1)
    assert ei.value.code == pkg.SIEVE_E_RANGE
    with pytest.raises(pkg.SieveError) as ei:
        sv.list(2 ** 32 - 10, 2 ** 32 + 10, elem_bytes=4,
                out=torch.empty(100, dtype=torch.int32, device="cuda"))
    assert ei.value.code == pkg.SIEVE_E_DTYPE
    assert sv.count(7, 7) == 0


@pytest.mark.parametrize("params", [
    dict(segment_bytes=8192, block_threads=256),
    dict(segment_bytes=32768, block_threads=1024, presieve_groups=1),
    dict(segment_bytes=131072, block_threads=1024),
    dict(segment_bytes=159744, block_threads=512, split_hits=64),
    dict(segment_bytes=65536, block_threads=512, presieve_groups=pkg.PRESIEVE_NONE),
    dict(segment_bytes=49152, block_threads=256, presieve_groups=3, split_hits=2048),
    dict(segment_bytes=16384, bucket_threshold=70000),          # most primes through buckets
    dict(segment_bytes=49152, bucket_threshold=pkg.BUCKET_NEVER),  # no bucket sieve
    dict(cofactor_skip=pkg.SKIP_ALL, split_hits=24),            # skip 5 | cofactor in tiles too
    dict(cofactor_skip=pkg.SKIP_NONE, bucket_threshold=70000, segment_bytes=16384),
    dict(cofactor_skip=pkg.SKIP_SPLIT, split_hits=64),          # skip on split items only
    dict(dense_hits=pkg.DENSE_NEVER),                           # no fixed-mask marking
    dict(dense_hits=40, split_hits=8, segment_bytes=8192),      # fixed-mask marking for most primes
    dict(dense_hits=2000, cofactor_skip=pkg.SKIP_ALL),          # fixed-mask beside the skip path
    dict(split_hits=8),                                         # dense lane counts up to 384
    dict(segment_bytes=159744, split_hits=8),                   # dense lane counts up to 1184
    # strips: primes carried from tile to tile in registers
    dict(strip_tiles=1),                                        # every tile starts afresh
    dict(strip_tiles=2, segment_bytes=8192),                    # many short strips
    dict(strip_tiles=7, segment_bytes=16384, block_threads=256),  # registers and fresh starts
    dict(strip_tiles=64, segment_bytes=8192, block_threads=512),  # longest strips
    dict(strip_tiles=3, segment_bytes=16384, bucket_threshold=70000),  # strips beside buckets
    dict(strip_tiles=5, segment_bytes=32768, cofactor_skip=pkg.SKIP_ALL, dense_hits=pkg.DENSE_NEVER),
])
def test_parameter_grid_parity(params):
    with pkg.Sieve(0, params) as s:
        s.base_primes(10 ** 6)
        for lo, hi in [(0, 3 * 10 ** 7 + 17), (10 ** 11 - 5 * 10 ** 6, 10 ** 11 + 7 * 10 ** 6)]:
            got = _u(s.list(lo, hi, elem_bytes=8), 8)
            want = oracle.primes(lo, hi, elem_bytes=8)
            assert_same_primes(got, want, (params, lo, hi))
            assert s.count(lo, hi) == len(want)


def test_base_primes_match_oracle(sv):
    # the resident set grows through the device list path
    with pkg.Sieve(0) as s:
        n = s.base_primes(10 ** 7)
        assert n == len(oracle.simple_primes(10 ** 7)) - 2  # primes >= 5
        lo, hi = 10 ** 13, 10 ** 13 + 10 ** 6
        assert s.count(lo, hi) == oracle.count(lo, hi)


@pytest.mark.parametrize("thr,slices", [(0, 0), (200_000, 0), (pkg.BUCKET_NEVER, 0),
                                        (0, pkg.BUCKET_EXACT), (0, pkg.BUCKET_TINY)])
def test_bucket_sieve_long_ranges_at_1e15(thr, slices):
    """Multi-tile ranges near 10^15 with primes up to 3.2e7: bucketed and
    per-tile paths agree with the oracle and with each other."""
    rng = np.random.default_rng(21)
    lo = (10 ** 15 - np.floor(10 ** rng.uniform(7, 14, 12))).astype(np.uint64)
    hi = lo + np.floor(10 ** rng.uniform(6, 7.7, 12)).astype(np.uint64)
    lo[0], hi[0] = 10 ** 15 - 3 * 10 ** 7, 10 ** 15  # many tiles, hi at the top
    mode = (np.arange(12) % 2).astype(np.uint8)
    with pkg.Sieve(0, dict(bucket_threshold=thr, bucket_slices=slices)) as s:
        s.ensure_base_for(int(hi.max()))
        cap = np.array([pkg.list_bound(int(a), int(b)) for a, b in zip(lo, hi)], dtype=np.uint64)
        off = np.concatenate([[0], np.cumsum(cap)[:-1]]).astype(np.uint64)
        out = torch.empty(int(cap.sum()), dtype=torch.int64, device="cuda")
        counts, status = s.list_batch(lo, hi, mode, out, off, cap, elem_bytes=8)
        host = _u(out, 8)
        for i in range(12):
            want = oracle.primes(int(lo[i]), int(hi[i]), elem_bytes=8)
            assert status[i] == 0 and int(counts[i]) == len(want), (thr, i)
            if mode[i]:
                assert np.array_equal(host[int(off[i]):int(off[i]) + len(want)], want), (thr, i)
        assert s.count(int(lo[0]), int(hi[0])) == int(counts[0])


@pytest.mark.parametrize("elem_bytes", [4, 8])
def test_list_output_at_address_with_bit31_set(sv, elem_bytes):
    """Output pointers whose low 32 bits are >= 2^31 (the kernels carry the
    output address in two 32-bit halves; neither half may be sign-extended)."""
    lo, hi = 10 ** 9, 10 ** 9 + 3 * 10 ** 6
    cap = pkg.list_bound(lo, hi)
    n_el = (1 << 31) // elem_bytes + cap + 1024
    big = torch.empty(n_el, dtype=torch.int32 if elem_bytes == 4 else torch.int64, device="cuda")
    base = big.data_ptr()
    # first element index whose address has bit 31 set in its low word
    k = 0
    while ((base + k * elem_bytes) & 0x80000000) == 0:
        k += (1 << 20) // elem_bytes
    assert k + cap <= n_el
    got = _u(sv.list(lo, hi, out=big[k:k + cap], elem_bytes=elem_bytes), elem_bytes).astype(np.uint64)
    assert np.array_equal(got, oracle.primes(lo, hi))
    del big


def test_top_of_domain_window():
    """Tiles above 2^62 (the wide remainder path) up to hi = 2^63: every
    wheel candidate of the window is classified by deterministic
    Miller-Rabin (exact below 3.3e24), and counts agree with the list."""
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    hi = 1 << 63
    lo = hi - (1 << 17)
    with pkg.Sieve(0) as s:
        s.ensure_base_for(hi)  # primes up to isqrt(2^63 - 1) = 3037000499
        got = _u(s.list(lo, hi, elem_bytes=8), 8)
        want = [n for n in range(lo | 1, hi, 2) if n % 3 and brute.is_prime_mr(n)]
        assert np.array_equal(got, np.array(want, dtype=np.uint64))
        mid = lo + (1 << 16) + 7
        assert s.count(lo, mid) + s.count(mid, hi) == len(want)
        assert s.count_batch([lo, mid], [mid, hi]).sum() == len(want)


def test_lds_probe_modes():
    """The LDS probe runs every mode; a conflict-free pattern is at least as
    fast as random words, and random words faster than one word per wave."""
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    rates = {m: pkg.probe_lds(m, iters=256, wg_per_cu=2)[0] for m in pkg.PROBE_MODES}
    assert all(r > 0 for r in rates.values())
    assert rates["or_linear"] >= 0.9 * rates["or_random"]
    assert rates["or_random"] > rates["or_same"]
