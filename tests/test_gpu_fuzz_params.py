"""Seeded random launch parameters against the oracle's stored results.

Each draw picks a tile size (8 KiB to 152 KiB), workgroup size and count,
split and dense thresholds, presieve groups, cofactor-5 skip mode, strip
length, bucket threshold and layout, and visit order, then counts all 4096
batch ranges (seed 0) and lists twelve of the listed ones.
Counts must equal the oracle's (tests/golden/batch4096_seed0.txt) and every
list must hash, chunk by chunk, to the oracle's digests.  Plane ends, item
splits and strip boundaries move with every draw, which is where a lost or
extra mark hides.
"""
import numpy as np
import pytest

from conftest import chunk_digests, golden_mismatch, read_golden_results

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
pkg = pytest.importorskip("paper_2310_17746_amd")
from paper_2310_17746_amd import workloads  # noqa: E402

DRAWS = 96


def _draw(rng):
    seg = int(rng.choice([8192, 12288, 16384, 20480, 28672, 36864, 45056, 53248, 61440, 77824, 98304,
                          131072, 155648]))
    nt = int(rng.choice([256, 512, 1024]))
    fit = max(1, (160 * 1024) // seg)
    p = dict(segment_bytes=seg, block_threads=nt, wg_per_cu=int(rng.integers(1, min(fit, 4) + 1)),
             split_hits=int(rng.choice([8, 16, 32, 64, 128, 256])),
             dense_hits=int(rng.choice([32, 64, 128, 256, 512, 1024, 4096, pkg.DENSE_NEVER])),
             presieve_groups=int(rng.choice([1, 2, 3, 4, 5, 6, pkg.PRESIEVE_NONE])),
             cofactor_skip=int(rng.choice([0, pkg.SKIP_ALL, pkg.SKIP_NONE, pkg.SKIP_SPLIT])),
             strip_tiles=int(rng.choice([0, 1, 2, 3, 7, 16, 64])),
             bucket_threshold=int(rng.choice([0, 0, pkg.BUCKET_NEVER, 32 * seg // 8, 200000])),
             bucket_slices=int(rng.choice([0, 0, pkg.BUCKET_EXACT, pkg.BUCKET_TINY])),
             visit_order=int(rng.integers(0, 3)))
    return p


@pytest.fixture(scope="module")
def batch():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    lo, hi, mode = workloads.batch_ranges(0)
    counts, chunks = read_golden_results("batch4096_seed0.txt")
    want = np.array([counts[i] for i in range(len(lo))], dtype=np.uint64)
    return lo, hi, mode, want, chunks


@pytest.mark.parametrize("draw", range(DRAWS))
def test_random_parameters(batch, draw):
    lo, hi, mode, want, chunks = batch
    rng = np.random.default_rng(1000 + draw)
    p = _draw(rng)
    sel = np.arange(len(lo))
    print("fuzz %d: %s" % (draw, p), flush=True)
    with pkg.Sieve(0, p) as s:
        s.ensure_base_for(int(hi[sel].max()))
        got = s.count_batch(lo[sel], hi[sel])
        bad = np.nonzero(got != want[sel])[0]
        assert len(bad) == 0, [(int(sel[i]), int(lo[sel[i]]), int(hi[sel[i]]), int(got[i]), int(want[sel[i]]))
                               for i in bad[:6]]
        small = [int(i) for i in sel if mode[i] and int(i) in chunks and want[i] <= 4 * 10 ** 6]
        listed = [small[int(k)] for k in rng.choice(len(small), 12, replace=False)]
        for i in listed:
            v = s.list(int(lo[i]), int(hi[i]), elem_bytes=8).cpu().numpy().view(np.uint64)
            msg = golden_mismatch(chunk_digests(v), chunks[i])
            assert msg is None, (i, int(lo[i]), int(hi[i]), msg)
