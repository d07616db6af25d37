"""The serving workload at its own shape: the 2000 seeded requests (seed 1:
lo log-uniform in [10^6, 10^14], length log-uniform in [10^4, 10^9], 30%
listed as uint64) with Poisson arrivals, and the count of [2, 10^12]
submitted at t = 0, served together as the benchmark serves them (64 GiB
output arena, default steps).

In the mix every count equals the oracle's (tests/golden/serve2000_seed1.txt)
and every listed request's primes, fetched one at a time, hash chunk by chunk
to the oracle's digests; the long job gives pi(10^12).  Alone (one plain call
per request on the same context once the server is gone) every count and
every list is the same as in the mix, element by element.  Pieces of some
requests near 10^14 run the bucket sieve inside the server's steps.
"""
import time
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest

from conftest import chunk_digests, golden_mismatch, read_golden_results

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
pkg = pytest.importorskip("paper_2310_17746_amd")
from paper_2310_17746_amd import workloads  # noqa: E402

LAMBDA = 4.0e4  # arrivals per second (about 0.8 of the measured saturated rate)


@pytest.mark.parametrize("overlap", [0, 1])
def test_serving_mix_full_shape(pi_table, overlap):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    lo, hi, mode, gaps = workloads.serving_requests(1)
    n = len(lo)
    want_count, want_chunks = read_golden_results("serve2000_seed1.txt")
    assert len(want_count) == n and set(want_chunks) <= set(np.nonzero(mode)[0].tolist())
    long_lo, long_hi = workloads.LONG_JOB
    s = pkg.Sieve(0)
    try:
        s.ensure_base_for(max(int(hi.max()), long_hi))
        print("serve: %d requests + [%d, %d) at %.0f req/s" % (n, long_lo, long_hi, LAMBDA), flush=True)
        mix_lists = {}
        digests = {}
        done = {}
        pool = ThreadPoolExecutor(16)
        with pkg.Server(s, out_budget_bytes=64 << 30, elem_bytes=8, overlap=overlap) as srv:
            t0 = srv.now_ns() + 2_000_000
            srv.submit(long_lo, long_hi, 0, n, at_ns=t0)
            arrivals = np.cumsum(gaps) / LAMBDA * 1e9
            for i in range(n):
                srv.submit(int(lo[i]), int(hi[i]), int(mode[i]), i, at_ns=t0 + int(arrivals[i]))
            t_end = time.time() + 240
            while len(done) < n + 1:
                assert time.time() < t_end, "serving run did not finish: %d of %d" % (len(done), n + 1)
                for c in srv.poll(4096, wait_ms=20):
                    done[c["tag"]] = c
                    if c["mode"] == 1 and c["status"] == 0:
                        t = srv.fetch(c["tag"], c["count"])  # device copy; frees the arena space
                        mix_lists[c["tag"]] = t
                        digests[c["tag"]] = pool.submit(
                            lambda h: chunk_digests(h.numpy().view(np.uint64)), t.cpu())
            st = srv.stats()
        print("serve: mix done, %d steps, %d with buckets" % (st["steps"], st["bucket_steps"]), flush=True)
        assert done[n]["status"] == 0 and done[n]["count"] == pi_table[10 ** 12]
        bad = [i for i in range(n) if done[i]["status"] != 0 or done[i]["count"] != want_count[i]]
        assert not bad, [(i, int(lo[i]), int(hi[i]), done[i]["status"], done[i]["count"], want_count[i])
                         for i in bad[:5]]
        for i, f in digests.items():
            m = golden_mismatch(f.result(), want_chunks.get(i, []))
            assert m is None, "request %d [%d, %d) in the mix: %s" % (i, int(lo[i]), int(hi[i]), m)
        pool.shutdown()
        assert st["bucket_steps"] > 0, "no serving step ran the bucket sieve"

        # alone: one plain call per request, same context
        for i in range(n):
            a, b = int(lo[i]), int(hi[i])
            assert s.count(a, b) == done[i]["count"], (i, a, b)
            if mode[i]:
                alone = s.list(a, b, elem_bytes=8)
                assert torch.equal(alone, mix_lists.pop(i)), (i, a, b)
                del alone
        print("serve: alone == mix for every request", flush=True)
    finally:
        s.close()
