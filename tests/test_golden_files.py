"""The stored oracle results of the full-size workloads (tests/golden/, written
by tests/golden/make_golden.py) are complete and agree with the oracle.

Structure: one count row per range or request, chunk rows exactly for the
listed ones, chunk sizes adding up to the count, chunks that follow each
other in value.  Agreement: a seeded sample of entries of each file is
recomputed by the oracle here (count, and for lists every chunk's digest and
end values); for the window, its first and last chunks are listed afresh and
nothing lies outside them."""
import numpy as np

import oracle
from conftest import chunk_digests, read_golden_results
from paper_2310_17746_amd import workloads

WINDOW = (10 ** 12, 10 ** 12 + 10 ** 10)


def _structure(counts, chunks, n, listed):
    assert sorted(counts) == list(range(n))
    assert set(chunks) <= set(listed)
    for i in listed:
        cs = chunks.get(i, [])
        assert sum(c[2] for c in cs) == counts[i], i
        for a, b in zip(cs, cs[1:]):
            assert a[1] < b[0]
        for c in cs:
            assert c[0] <= c[1] and len(c[3]) == 32


def _recompute(lo, hi, mode, counts, chunks, idx):
    for i in idx:
        a, b = int(lo[i]), int(hi[i])
        if mode[i]:
            v = oracle.primes(a, b, elem_bytes=8)
            assert len(v) == counts[i], i
            assert chunk_digests(v) == chunks.get(i, []), i
        else:
            assert oracle.count(a, b) == counts[i], i


def _sample(lo, hi, k, seed, max_len):
    short = np.nonzero((hi - lo) <= max_len)[0]
    return np.random.default_rng(seed).choice(short, k, replace=False)


def test_batch_results_file():
    lo, hi, mode = workloads.batch_ranges(0)
    counts, chunks = read_golden_results("batch4096_seed0.txt")
    _structure(counts, chunks, len(lo), np.nonzero(mode)[0].tolist())
    _recompute(lo, hi, mode, counts, chunks, _sample(lo, hi, 12, 7, 10 ** 6))


def test_serving_results_file():
    lo, hi, mode, _ = workloads.serving_requests(1)
    counts, chunks = read_golden_results("serve2000_seed1.txt")
    _structure(counts, chunks, len(lo), np.nonzero(mode)[0].tolist())
    _recompute(lo, hi, mode, counts, chunks, _sample(lo, hi, 12, 8, 10 ** 6))
    # a request with more than one chunk: its first chunk's span, listed afresh
    big = [i for i, cs in chunks.items() if len(cs) > 1]
    if big:
        f, l, n, d = chunks[big[0]][0]
        v = oracle.primes(f, l + 1, elem_bytes=8)
        assert chunk_digests(v) == [(f, l, n, d)]


def test_window_results_file():
    counts, chunks = read_golden_results("window_1e12_1e10.txt")
    _structure(counts, chunks, 1, [0])
    cs = chunks[0]
    assert cs[0][0] >= WINDOW[0] and cs[-1][1] < WINDOW[1]
    for k in (0, len(cs) - 1):  # the first and the last chunk, listed afresh
        f, l, n, d = cs[k]
        v = oracle.primes(f, l + 1, elem_bytes=8)
        assert chunk_digests(v) == [(f, l, n, d)]
    # no prime between the window start and the first chunk, or after the last
    assert oracle.count(WINDOW[0], cs[0][0]) == 0 and oracle.count(cs[-1][1] + 1, WINDOW[1]) == 0
