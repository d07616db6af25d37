"""Stream-ordered calls: with a stream, sieve_list / sieve_count_batch /
sieve_list_batch enqueue their job and return; the host outputs are written
when the stream reaches the end of the job.  Dependent torch work queued on
the same stream sees the finished list; results are bit-exact against the
oracle after one synchronisation; jobs of one context on two streams are
ordered; a job that takes the bucket sieve waits and is still exact."""
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
    s = pkg.Sieve(0)
    s.base_primes(10 ** 7)
    yield s
    s.close()


def test_list_on_torch_stream_then_dependent_work(sv):
    lo, hi = 10 ** 12, 10 ** 12 + 3 * 10 ** 8
    st = torch.cuda.Stream()
    with torch.cuda.stream(st):
        out = torch.full((pkg.list_bound(lo, hi),), -1, dtype=torch.int64, device="cuda")
        r = sv.list_async(lo, hi, out, 8, st)
        # dependent work on the same stream: a copy and a reduction of the list buffer
        copy = out.clone()
        positive = (copy > 0).sum()
    st.synchronize()
    want = oracle.primes(lo, hi, elem_bytes=8)
    n = r.count
    assert n == len(want)
    got = copy[:n].cpu().numpy().view(np.uint64)
    assert np.array_equal(got, want)
    assert int(positive) == n  # the rest of the buffer still holds the -1 fill
    assert bool((copy[n:] == -1).all())


def test_count_batch_returns_before_the_job_ends(sv):
    lo = np.array([2, 10 ** 10, 10 ** 11 - 10 ** 9, 7], dtype=np.uint64)
    hi = np.array([10 ** 11 + 1, 10 ** 10 + 10 ** 9, 10 ** 11, 7], dtype=np.uint64)
    st = torch.cuda.Stream()
    counts = sv.count_batch(lo, hi, stream=st, sync=False)
    pending = not st.query()  # about 10 ms of sieving was just enqueued
    st.synchronize()
    assert pending
    assert counts[0] == 4118054813 and counts[3] == 0
    assert counts[1] == oracle.count(10 ** 10, 10 ** 10 + 10 ** 9)
    assert counts[2] == oracle.count(10 ** 11 - 10 ** 9, 10 ** 11)


def test_two_streams_one_context(sv):
    a = torch.cuda.Stream()
    b = torch.cuda.Stream()
    lo, hi = 10 ** 9, 10 ** 9 + 10 ** 8
    with torch.cuda.stream(a):
        out_a = torch.empty(pkg.list_bound(lo, hi), dtype=torch.int64, device="cuda")
    with torch.cuda.stream(b):
        out_b = torch.empty(pkg.list_bound(lo + 5, hi + 5), dtype=torch.int64, device="cuda")
    ra = sv.list_async(lo, hi, out_a, 8, a)
    rb = sv.list_async(lo + 5, hi + 5, out_b, 8, b)
    cb = sv.count_batch([lo], [hi], stream=b, sync=False)
    a.synchronize()
    b.synchronize()
    want = oracle.primes(lo, hi + 5, elem_bytes=8)
    wa, wb = want[want < hi], want[want >= lo + 5]
    assert np.array_equal(ra.primes().cpu().numpy().view(np.uint64), wa)
    assert np.array_equal(rb.primes().cpu().numpy().view(np.uint64), wb)
    assert int(cb[0]) == len(wa)


def test_list_batch_stream_ordered_and_capacity(sv):
    lo = np.array([10 ** 8, 10 ** 9, 3], dtype=np.uint64)
    hi = np.array([10 ** 8 + 10 ** 6, 10 ** 9 + 10 ** 6, 100], dtype=np.uint64)
    mode = np.array([1, 1, 1], dtype=np.uint8)
    cap = np.array([pkg.list_bound(int(a), int(b)) for a, b in zip(lo, hi)], dtype=np.uint64)
    cap[2] = 3  # too small: that range reports SIEVE_E_CAPACITY, the others are unaffected
    off = np.concatenate([[0], np.cumsum(cap)[:-1]]).astype(np.uint64)
    st = torch.cuda.Stream()
    with torch.cuda.stream(st):
        out = torch.empty(int(cap.sum()), dtype=torch.int64, device="cuda")
    counts, status = sv.list_batch(lo, hi, mode, out, off, cap, stream=st, sync=False)
    st.synchronize()
    assert list(status) == [0, 0, pkg.SIEVE_E_CAPACITY]
    host = out.cpu().numpy().view(np.uint64)
    for i in range(2):
        want = oracle.primes(int(lo[i]), int(hi[i]), elem_bytes=8)
        assert int(counts[i]) == len(want)
        assert np.array_equal(host[int(off[i]):int(off[i]) + len(want)], want)
    assert int(counts[2]) == oracle.count(3, 100)


def test_bucket_job_with_a_stream_is_exact():
    # ranges near 10^15 of several tiles take the bucket sieve: the call waits
    with pkg.Sieve(0) as s:
        lo, hi = 10 ** 15, 10 ** 15 + 4 * 10 ** 7
        s.ensure_base_for(hi)
        st = torch.cuda.Stream()
        with torch.cuda.stream(st):
            out = torch.empty(pkg.list_bound(lo, hi), dtype=torch.int64, device="cuda")
        r = s.list_async(lo, hi, out, 8, st)
        st.synchronize()
        assert np.array_equal(r.primes().cpu().numpy().view(np.uint64), oracle.primes(lo, hi, elem_bytes=8))
