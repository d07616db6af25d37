"""Serving engine on the GPU: every request's result in the mix equals its
result alone (bit-exact) and the oracle's; admission by output memory,
cancellation and scheduled arrivals behave as documented."""
import time
from math import isqrt

import numpy as np
import pytest

import oracle
from conftest import read_golden

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
pkg = pytest.importorskip("paper_2310_17746_amd")


def _u(t):
    return t.cpu().numpy().view(np.uint64)


@pytest.fixture(scope="module")
def sv():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    s = pkg.Sieve(0)
    s.base_primes(10 ** 6)
    yield s
    s.close()


def _drain(srv, n, timeout_s=120):
    got = {}
    t_end = time.time() + timeout_s
    while len(got) < n and time.time() < t_end:
        for c in srv.poll(4096, wait_ms=50):
            got[c["tag"]] = c
    assert len(got) == n, "server did not finish: %d of %d" % (len(got), n)
    return got


@pytest.mark.parametrize("overlap", [0, 1])
def test_alone_vs_mix_with_long_job(sv, overlap):
    pi = {int(x): int(v) for x, v in read_golden("pi_values.txt")}
    rng = np.random.default_rng(5)
    n = 120
    lo = np.floor(10 ** rng.uniform(0, 11.5, n)).astype(np.uint64)
    hi = lo + np.floor(10 ** rng.uniform(0, 7, n)).astype(np.uint64)
    mode = (rng.random(n) < 0.4).astype(int)
    lo[:4] = [0, 2, 3, 10 ** 6]
    hi[:4] = [0, 4, 3, 10 ** 6 + 1]
    alone_c = [sv.count(int(a), int(b)) for a, b in zip(lo, hi)]
    alone_l = {i: _u(sv.list(int(lo[i]), int(hi[i]), elem_bytes=8)) for i in range(n) if mode[i]}
    long_tag = 10 ** 6
    with pkg.Server(sv, out_budget_bytes=512 << 20, step_tiles=96, quantum_tiles=4, overlap=overlap) as srv:
        srv.submit(2, 10 ** 10 + 1, 0, long_tag)
        for i in range(n):
            srv.submit(int(lo[i]), int(hi[i]), int(mode[i]), i)
        got = _drain(srv, n + 1)
        assert got[long_tag]["status"] == 0 and got[long_tag]["count"] == pi[10 ** 10]
        for i in range(n):
            c = got[i]
            assert c["status"] == 0, (i, c)
            assert c["count"] == alone_c[i], (i, int(lo[i]), int(hi[i]))
            if mode[i]:
                lst = _u(srv.fetch(i, c["count"]))
                assert np.array_equal(lst, alone_l[i]), i
                assert np.array_equal(lst, oracle.primes(int(lo[i]), int(hi[i]), elem_bytes=8)), i
        # the long job shares the device: most short requests finish first
        short_done = np.array([got[i]["t_done_ns"] for i in range(n)])
        assert np.mean(short_done < got[long_tag]["t_done_ns"]) > 0.9
        st = srv.stats()
        assert st["completed"] == n + 1 and st["active"] == 0
        assert (st["overlap_steps"] > 0) == bool(overlap)
        assert 0 < st["busy_ns"] <= st["elapsed_ns"]


@pytest.mark.parametrize("overlap", [0, 1])
def test_cancel_long_job(sv, overlap):
    with pkg.Server(sv, step_tiles=32, quantum_tiles=2, overlap=overlap) as srv:
        srv.submit(2, 10 ** 11 + 1, 0, 7)
        time.sleep(0.05)
        assert srv.cancel(7) == 0
        (c,) = _drain(srv, 1).values()
        assert c["status"] == pkg.SIEVE_E_CANCELLED
        assert srv.cancel(7) == pkg.SIEVE_E_INVAL  # no longer live


def test_admission_by_output_budget(sv):
    lo, hi = 10 ** 9, 10 ** 9 + 2 * 10 ** 6
    bound = pkg.list_bound(lo, hi) * 8
    budget = (bound * 3) // 2                 # one list request fits, not two
    with pkg.Server(sv, out_budget_bytes=budget) as srv:
        srv.submit(0, 10 ** 8, 1, 99)         # bound exceeds the whole budget
        srv.submit(lo, hi, 1, 1)
        srv.submit(lo, hi, 1, 2)
        first = {}
        t_end = time.time() + 60
        while len(first) < 2 and time.time() < t_end:
            for c in srv.poll(16, wait_ms=50):
                first[c["tag"]] = c
        assert first[99]["status"] == pkg.SIEVE_E_NOMEM
        assert first[1]["status"] == 0
        time.sleep(0.2)
        assert 2 not in first and srv.stats()["queued"] == 1  # waits for memory
        want = oracle.primes(lo, hi, elem_bytes=8)
        assert np.array_equal(_u(srv.fetch(1, first[1]["count"])), want)  # frees its space
        (c2,) = _drain(srv, 1).values()
        assert c2["tag"] == 2 and c2["status"] == 0 and c2["t_admit_ns"] > first[1]["t_done_ns"]
        assert np.array_equal(_u(srv.fetch(2, c2["count"])), want)


def test_scheduled_arrivals(sv):
    with pkg.Server(sv) as srv:
        t0 = srv.now_ns()
        arr = [t0 + k * 20_000_000 for k in range(5)]  # every 20 ms
        for k, t in enumerate(arr):
            srv.submit(10 ** 10, 10 ** 10 + 10 ** 6, 0, k, at_ns=t)
        got = _drain(srv, 5)
        want = oracle.count(10 ** 10, 10 ** 10 + 10 ** 6)
        for k in range(5):
            c = got[k]
            assert c["count"] == want
            assert c["t_arrival_ns"] == arr[k] and c["t_admit_ns"] >= arr[k] and c["t_done_ns"] >= c["t_admit_ns"]


@pytest.mark.parametrize("overlap", [0, 1])
def test_base_primes_grow_while_steps_run(overlap):
    """A fresh context with small base primes: requests arrive that need more
    of them while earlier steps are on the device (with overlap, one is still
    in flight when the store is re-installed).  Every count is the oracle's."""
    reqs = [(10 ** 6, 10 ** 6 + 10 ** 6), (10 ** 10, 10 ** 10 + 10 ** 6), (10 ** 12, 10 ** 12 + 10 ** 6),
            (10 ** 14, 10 ** 14 + 10 ** 6), (2, 10 ** 9 + 1), (10 ** 15, 10 ** 15 + 10 ** 5)]
    with pkg.Sieve(0) as s:
        s.base_primes(1 << 16)
        with pkg.Server(s, step_tiles=64, quantum_tiles=4, overlap=overlap) as srv:
            for i, (lo, hi) in enumerate(reqs):
                srv.submit(lo, hi, 0, i)
            got = _drain(srv, len(reqs))
        for i, (lo, hi) in enumerate(reqs):
            assert got[i]["status"] == 0 and got[i]["count"] == oracle.count(lo, hi), (i, lo, hi)
        assert s.base_limit >= max(isqrt(hi - 1) for _, hi in reqs)



@pytest.mark.parametrize("overlap", [0, 1])
def test_submit_into_caller_buffers(sv, overlap):
    """sieve_submit_out: lists written straight into caller-owned tensors,
    beside arena lists and a long count; a buffer one element short reports
    SIEVE_E_CAPACITY with the full count."""
    reqs = [(10 ** 9, 10 ** 9 + 2 * 10 ** 6), (10 ** 11 - 5 * 10 ** 6, 10 ** 11 + 10 ** 6),
            (3, 5 * 10 ** 5), (10 ** 10, 10 ** 10 + 4 * 10 ** 7)]
    want = [oracle.primes(lo, hi, elem_bytes=8) for lo, hi in reqs]
    outs = [torch.full((len(w) + 3,), -1, dtype=torch.int64, device="cuda") for w in want]
    short = torch.empty(len(want[3]) - 1, dtype=torch.int64, device="cuda")
    with pkg.Server(sv, step_tiles=64, quantum_tiles=4, overlap=overlap) as srv:
        srv.submit(2, 10 ** 10 + 1, 0, 100)
        for i, (lo, hi) in enumerate(reqs[:3]):
            srv.submit(lo, hi, 1, i, out=outs[i])
        srv.submit(reqs[3][0], reqs[3][1], 1, 3, out=short)
        srv.submit(reqs[0][0], reqs[0][1], 1, 50)  # the same range through the arena
        got = _drain(srv, 6)
        for i in range(3):
            assert got[i]["status"] == 0 and got[i]["count"] == len(want[i]), i
            host = outs[i].cpu().numpy().view(np.uint64)
            assert np.array_equal(host[:len(want[i])], want[i]), i
            assert np.all(outs[i][len(want[i]):].cpu().numpy() == -1)  # nothing past the list
        assert got[3]["status"] == pkg.SIEVE_E_CAPACITY and got[3]["count"] == len(want[3])
        assert got[50]["status"] == 0
        assert np.array_equal(_u(srv.fetch(50, got[50]["count"])), want[0])
        assert got[100]["status"] == 0 and got[100]["count"] == 455052511


@pytest.mark.parametrize("overlap,slices", [(0, 0), (1, 0), (0, "tiny"), (0, "exact"), (0, "s52"), (0, "s76")])
def test_resident_bucket_walks(overlap, slices):
    """Requests cut into many two-tile pieces whose large primes take the
    bucket sieve: each piece resumes its request's bucket walks from the state
    the previous piece left on the device (Sec. 2.4's incremental state) and
    stores its own.  Counts and lists equal the oracle's and those of a server
    that restarts every walk, and the resumed path ran.  With one-entry
    estimated slices every bucket job overflows and runs again in the exact
    layout, after the estimated pass already stored the end state: the re-run
    must resume from the same source."""
    reqs = [(5 * 10 ** 13 + 7, 5 * 10 ** 13 + 73_000_000, 0),
            (10 ** 14 - 30_000_000, 10 ** 14 + 12_000_000, 1),
            (2 * 10 ** 13, 2 * 10 ** 13 + 50_000_001, 0),
            (9 * 10 ** 13, 9 * 10 ** 13 + 10 ** 6, 1),
            (7 * 10 ** 13 + 1, 7 * 10 ** 13 + 40_000_000, 1)]
    want_c = [oracle.count(lo, hi) for lo, hi, _ in reqs]
    want_l = {i: oracle.primes(lo, hi, elem_bytes=8) for i, (lo, hi, m) in enumerate(reqs) if m}
    results = {}
    prm = {0: {}, "tiny": dict(bucket_slices=pkg.BUCKET_TINY), "exact": dict(bucket_slices=pkg.BUCKET_EXACT),
           # the autotuner's smaller tiles: more primes go through the bucket sieve
           "s52": dict(segment_bytes=53248, block_threads=512, wg_per_cu=3),
           "s76": dict(segment_bytes=77824, block_threads=512, wg_per_cu=2)}[slices]
    with pkg.Sieve(0, prm) as s:
        s.base_primes(isqrt(max(hi for _, hi, _ in reqs)) + 1)
        for restart in (0, 1):
            print("resident walks: overlap %d slices %s restart %d" % (overlap, slices, restart), flush=True)
            with pkg.Server(s, step_tiles=8, quantum_tiles=2, overlap=overlap, restart_walks=restart,
                            out_budget_bytes=256 << 20) as srv:
                for i, (lo, hi, m) in enumerate(reqs):
                    srv.submit(lo, hi, m, i)
                got = _drain(srv, len(reqs))
                lists = {i: _u(srv.fetch(i, got[i]["count"])) for i in want_l}
                st = srv.stats()
            for i in range(len(reqs)):
                assert got[i]["status"] == 0 and got[i]["count"] == want_c[i], (restart, i, reqs[i])
            for i, w in want_l.items():
                assert np.array_equal(lists[i], w), (restart, i, reqs[i])
            assert st["bucket_steps"] > 0
            if restart:
                assert st["resumed_walks"] == 0 and st["walk_bytes"] == 0
            else:
                assert st["walk_bytes"] > 0
                if not overlap:
                    assert st["resumed_walks"] > 20
            results[restart] = ({i: got[i]["count"] for i in got}, lists)
    assert results[0][0] == results[1][0]
