"""Batched persistent form on the full 4096-range workload (seed 0: lo
log-uniform in [10^6, 10^15], length log-uniform in [10^3, 10^8], half listed
as uint64).

Every count equals the oracle's and every one of the 2048 listed ranges
hashes to the oracle's SHA-256 (tests/golden/batch4096_seed0.txt, written by
the oracle).  The same ranges run one plain call each give identical counts
and identical lists, element by element, and a replay of the captured graph
gives the same output again.
"""
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest

from conftest import chunk_digests, golden_mismatch, read_golden_results

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
pkg = pytest.importorskip("paper_2310_17746_amd")
from paper_2310_17746_amd import workloads  # noqa: E402


@pytest.fixture(scope="module")
def batch():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    lo, hi, mode = workloads.batch_ranges(0)
    counts, chunks = read_golden_results("batch4096_seed0.txt")
    assert len(counts) == len(lo) and set(chunks) <= set(np.nonzero(mode)[0].tolist())
    want = np.array([counts[i] for i in range(len(lo))], dtype=np.uint64)
    return lo, hi, mode, want, chunks


def _run(s, lo, hi, mode):
    cap = np.array([pkg.list_bound(int(a), int(b)) if m else 0 for a, b, m in zip(lo, hi, mode)],
                   dtype=np.uint64)
    off = np.concatenate([[0], np.cumsum(cap)[:-1]]).astype(np.uint64)
    out = torch.empty(int(cap.sum()) + 1, dtype=torch.int64, device="cuda")
    counts, status = s.list_batch(lo, hi, mode, out, off, cap, elem_bytes=8)
    return counts, status, out, off


@pytest.mark.parametrize("use_graph", [0, 1])
def test_full_batch_counts_and_lists(batch, use_graph):
    lo, hi, mode, want, chunks = batch
    print("batch: 4096 ranges, use_graph=%d" % use_graph, flush=True)
    with pkg.Sieve(0, dict(use_graph=use_graph)) as s:
        s.ensure_base_for(int(hi.max()))
        counts, status, out, off = _run(s, lo, hi, mode)
        assert np.all(status == 0)
        bad = np.nonzero(counts != want)[0]
        assert len(bad) == 0, [(int(lo[i]), int(hi[i]), int(counts[i]), int(want[i])) for i in bad[:5]]
        host = out.cpu().numpy().view(np.uint64)
        lst = np.nonzero(mode)[0]

        def check(i):
            o, c = int(off[i]), int(counts[i])
            return i, golden_mismatch(chunk_digests(host[o:o + c]), chunks.get(int(i), []))

        with ThreadPoolExecutor(16) as ex:
            for i, m in ex.map(check, lst):
                assert m is None, "range %d [%d, %d): %s" % (i, int(lo[i]), int(hi[i]), m)
        if use_graph:
            # a second replay of the same graph gives the same results
            counts2, status2, out2, _ = _run(s, lo, hi, mode)
            assert np.array_equal(counts2, counts) and np.all(status2 == 0)
            assert torch.equal(out2[: out.numel()], out)


def test_batch_equals_per_range_calls(batch):
    lo, hi, mode, want, _ = batch
    with pkg.Sieve(0) as s:
        s.ensure_base_for(int(hi.max()))
        counts, status, out, off = _run(s, lo, hi, mode)
        assert np.all(status == 0)
        for i in range(len(lo)):
            a, b = int(lo[i]), int(hi[i])
            assert s.count(a, b) == int(want[i]) == int(counts[i]), (i, a, b)
            if mode[i]:
                o, c = int(off[i]), int(counts[i])
                got = s.list(a, b, elem_bytes=8)
                assert torch.equal(got, out[o:o + c]), (i, a, b)
