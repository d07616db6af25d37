"""Split tiles (a tile's primes spread over several workgroups that meet in a
global copy of the planes) together with the other job features: captured
graphs replayed across jobs whose split layouts differ, piecewise jobs
under a small bucket budget, and capacity errors in list mode.  Bit-exact
against the oracle."""
import numpy as np
import pytest

import oracle

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
pkg = pytest.importorskip("paper_2310_17746_amd")

E14, E15 = 10 ** 14, 10 ** 15


def _u64(t):
    return t.cpu().numpy().view(np.uint64)


@pytest.fixture(scope="module")
def gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _want(lo, hi):
    return [oracle.primes(int(a), int(b), elem_bytes=8, threads=4) for a, b in zip(lo, hi)]


def _check_list(s, lo, hi, mode, want):
    cap = np.array([pkg.list_bound(int(a), int(b)) if m else 0 for a, b, m in zip(lo, hi, mode)],
                   dtype=np.uint64)
    off = np.concatenate([[0], np.cumsum(cap)[:-1]]).astype(np.uint64)
    out = torch.zeros(int(cap.sum()) + 1, dtype=torch.int64, device="cuda")
    counts, status = s.list_batch(lo, hi, mode, out, off, cap, elem_bytes=8)
    host = _u64(out)
    for i in range(len(lo)):
        assert int(counts[i]) == len(want[i]) and status[i] == 0, i
        if mode[i]:
            o = int(off[i])
            assert np.array_equal(host[o:o + len(want[i])], want[i]), i


def test_graph_replay_across_split_layouts(gpu):
    # three jobs in turn: split parts of different sizes and counts, one
    # without any split tile; each captured and replayed
    jobs = [
        (np.array([E15 + 7, 3 * E14 + 11], dtype=np.uint64), np.array([E15 + 200007, 3 * E14 + 900011], dtype=np.uint64)),
        (np.array([10 ** 9, 5 * E14], dtype=np.uint64), np.array([10 ** 9 + 4 * 10 ** 6, 5 * E14 + 60000], dtype=np.uint64)),
        (np.array([12345, 10 ** 11], dtype=np.uint64), np.array([10 ** 6, 10 ** 11 + 10 ** 6], dtype=np.uint64)),
    ]
    with pkg.Sieve(0, dict(use_graph=1)) as s:
        s.ensure_base_for(E15 + 10 ** 6)
        for rep in range(2):
            for lo, hi in jobs:
                want = _want(lo, hi)
                assert np.array_equal(s.count_batch(lo, hi), np.array([len(w) for w in want], dtype=np.uint64))
                _check_list(s, lo, hi, np.array([1, 0], dtype=np.uint8), want)
                torch.cuda.synchronize()


def test_pieces_with_split_tiles(gpu):
    # a 1 MiB bucket budget cuts the long bucket range into pieces; the
    # heavy single-tile ranges beside it are split
    lo = np.array([E14 - 30 * 10 ** 6, E15 - 10 ** 5, 7 * E14], dtype=np.uint64)
    hi = np.array([E14 + 30 * 10 ** 6, E15 + 10 ** 5, 7 * E14 + 5 * 10 ** 5], dtype=np.uint64)
    want = _want(lo, hi)
    with pkg.Sieve(0, dict(bucket_mem_mb=1)) as s:
        s.ensure_base_for(int(hi.max()))
        assert np.array_equal(s.count_batch(lo, hi), np.array([len(w) for w in want], dtype=np.uint64))
        _check_list(s, lo, hi, np.array([1, 1, 1], dtype=np.uint8), want)


def test_split_tile_capacity_error(gpu):
    lo, hi = E15, E15 + 300000
    n_true = oracle.count(lo, hi)
    with pkg.Sieve(0) as s:
        s.ensure_base_for(hi)
        out = torch.zeros(max(n_true - 1, 1), dtype=torch.int64, device="cuda")
        counts, status = s.list_batch(np.array([lo, 2], dtype=np.uint64), np.array([hi, 1000], dtype=np.uint64),
                                      np.array([1, 1], dtype=np.uint8), out,
                                      np.array([0, 0], dtype=np.uint64),
                                      np.array([n_true - 1, 0], dtype=np.uint64), elem_bytes=8)
        assert int(counts[0]) == n_true and status[0] == pkg.SIEVE_E_CAPACITY
        assert int(counts[1]) == 168 and status[1] == pkg.SIEVE_E_CAPACITY
