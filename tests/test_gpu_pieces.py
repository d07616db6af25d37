"""Jobs larger than the bucket-memory budget run as tile-aligned pieces.

With a 1 MiB budget and the bucket sieve on every multi-tile range, long
ranges are cut into many pieces; counts, lists, mixed batches and the
capacity status must match the oracle exactly as for a single job.
"""
import numpy as np
import pytest

import oracle

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
pkg = pytest.importorskip("paper_2310_17746_amd")


@pytest.fixture(scope="module")
def sv():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    s = pkg.Sieve(0, dict(bucket_threshold=65536, bucket_mem_mb=1))
    s.base_primes(1 << 21)
    yield s
    s.close()


def test_pieces_count_long_range(sv):
    lo, hi = 10 ** 12 - 777, 10 ** 12 + 2 * 10 ** 9 + 5
    assert sv.count(lo, hi) == oracle.count(lo, hi)


def test_pieces_list_long_range(sv):
    lo, hi = 10 ** 12 + 11, 10 ** 12 + 3 * 10 ** 8 + 1
    got = sv.list(lo, hi, elem_bytes=8).cpu().numpy().view(np.uint64)
    assert np.array_equal(got, oracle.primes(lo, hi))


def test_pieces_mixed_batch_with_capacity(sv):
    lo = np.array([10 ** 12, 5, 10 ** 12 + 5 * 10 ** 8, 10 ** 13, 7 * 10 ** 11, 10 ** 12 + 9 * 10 ** 8],
                  dtype=np.uint64)
    hi = lo + np.array([4 * 10 ** 8, 10 ** 6, 2 * 10 ** 8, 10 ** 4, 3 * 10 ** 8, 10 ** 8], dtype=np.uint64)
    mode = np.array([1, 1, 0, 1, 1, 1], dtype=np.uint8)
    sv.ensure_base_for(int(hi.max()))
    want = [oracle.primes(int(a), int(b)) for a, b in zip(lo, hi)]
    cap = np.array([pkg.list_bound(int(a), int(b)) for a, b in zip(lo, hi)], dtype=np.uint64)
    cap[4] = len(want[4]) - 1  # one element short: SIEVE_E_CAPACITY, count still exact
    off = np.concatenate([[0], np.cumsum(cap)[:-1]]).astype(np.uint64)
    out = torch.zeros(int(cap.sum()) + 1, dtype=torch.int64, device="cuda")
    counts, status = sv.list_batch(lo, hi, mode, out, off, cap, elem_bytes=8)
    o = out.cpu().numpy().view(np.uint64)
    for i in range(len(lo)):
        assert int(counts[i]) == len(want[i]), i
        if i == 4:
            assert status[i] == pkg.SIEVE_E_CAPACITY
            continue
        assert status[i] == pkg.SIEVE_OK, i
        if mode[i]:
            a = int(off[i])
            assert np.array_equal(o[a:a + len(want[i])], want[i]), i


def test_pieces_match_single_job():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    lo = np.array([10 ** 12, 3 * 10 ** 12 + 1], dtype=np.uint64)
    hi = lo + np.array([10 ** 9, 7 * 10 ** 8], dtype=np.uint64)
    with pkg.Sieve(0, dict(bucket_threshold=65536)) as whole, \
            pkg.Sieve(0, dict(bucket_threshold=65536, bucket_mem_mb=2)) as pieces:
        whole.ensure_base_for(int(hi.max()))
        pieces.ensure_base_for(int(hi.max()))
        assert np.array_equal(whole.count_batch(lo, hi), pieces.count_batch(lo, hi))
