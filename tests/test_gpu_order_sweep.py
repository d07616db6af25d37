"""Parity sweep over the order in which workgroups take tiles (costly
first, reversed, shuffled) and over launch shapes and bucket thresholds.
Every mark of a tile is made by the workgroup that holds it (or, for a
split tile, meets in its global planes), so a race or a lost mark would
show up as a count or list mismatch in some cell.  Bit-exact against the
oracle."""
import numpy as np
import pytest

import oracle

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
pkg = pytest.importorskip("paper_2310_17746_amd")


@pytest.fixture(scope="module")
def case():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    rng = np.random.default_rng(31)
    n = 96
    lo = np.floor(10 ** rng.uniform(6, 15, n)).astype(np.uint64)
    hi = lo + np.floor(10 ** rng.uniform(3, 7, n)).astype(np.uint64)
    lo[:4] = [2, 10 ** 15, 10 ** 12, 5]          # the start of the domain, empty and
    hi[:4] = [3 * 10 ** 6, 10 ** 15, 10 ** 12 + 1, 6]  # one-value ranges among the rest
    mode = (rng.random(n) < 0.5).astype(np.uint8)
    want = [oracle.primes(int(a), int(b), elem_bytes=8, threads=4) for a, b in zip(lo, hi)]
    return lo, hi, mode, want


@pytest.mark.parametrize("order", [pkg.VISIT_COSTLY_FIRST, pkg.VISIT_REVERSED, pkg.VISIT_SHUFFLED])
@pytest.mark.parametrize("params", [{}, dict(segment_bytes=32768, block_threads=256, wg_per_cu=4),
                                    dict(bucket_threshold=425984)])
def test_visit_order_sweep(case, order, params):
    lo, hi, mode, want = case
    with pkg.Sieve(0, dict(params, visit_order=order)) as s:
        s.ensure_base_for(int(hi.max()))
        assert np.array_equal(s.count_batch(lo, hi), np.array([len(w) for w in want], dtype=np.uint64))
        cap = np.array([pkg.list_bound(int(a), int(b)) if m else 0 for a, b, m in zip(lo, hi, mode)],
                       dtype=np.uint64)
        off = np.concatenate([[0], np.cumsum(cap)[:-1]]).astype(np.uint64)
        out = torch.zeros(int(cap.sum()) + 1, dtype=torch.int64, device="cuda")
        counts, status = s.list_batch(lo, hi, mode, out, off, cap, elem_bytes=8)
        host = out.cpu().numpy().view(np.uint64)
        for i in range(len(lo)):
            assert int(counts[i]) == len(want[i]) and status[i] == 0, (order, params, i)
            if mode[i]:
                o = int(off[i])
                assert np.array_equal(host[o:o + len(want[i])], want[i]), (order, params, i)


def test_visit_order_rejects_unknown():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    with pytest.raises(pkg.SieveError):
        pkg.Sieve(0, dict(visit_order=3))
