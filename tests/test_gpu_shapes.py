"""Every launch shape the autotuner may pick gives the oracle's counts on the
whole 4096-range batch (seed 0) and on the headline count, range by range.

The shapes differ in the kernel variant they select (four or six waves per
SIMD, 32 or 8 carried primes per thread), tile size, strip length, the
cofactor-5 skip mode that goes with the variant, and the bucket threshold.
A mismatch names the shape, the first differing ranges and whether the same
range alone (one call, same shape) is right.
"""
import numpy as np
import pytest

from conftest import read_golden_results

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
pkg = pytest.importorskip("paper_2310_17746_amd")
from paper_2310_17746_amd import autotune, workloads  # noqa: E402

PI_1E11 = 4118054813

SHAPES = [{}] + autotune.GRIDS["batch"] + [g for g in autotune.GRIDS["count"] if g.get("strip_tiles")]


@pytest.fixture(scope="module")
def batch():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    lo, hi, _ = workloads.batch_ranges(0)
    counts, _ = read_golden_results("batch4096_seed0.txt")
    want = np.array([counts[i] for i in range(len(lo))], dtype=np.uint64)
    return lo, hi, want


@pytest.mark.parametrize("params", SHAPES, ids=lambda p: ",".join("%s=%s" % kv for kv in sorted(p.items())) or "default")
def test_shape_counts_match_oracle(batch, params):
    lo, hi, want = batch
    print("shapes: %s" % params, flush=True)
    with pkg.Sieve(0, params) as s:
        s.ensure_base_for(int(hi.max()))
        got = s.count_batch(lo, hi)
        bad = np.nonzero(got != want)[0]
        detail = []
        for i in bad[:8]:
            alone = s.count(int(lo[i]), int(hi[i]))
            detail.append((int(i), int(lo[i]), int(hi[i]), int(got[i]), int(want[i]), alone))
        assert len(bad) == 0, "%d ranges differ; (i, lo, hi, batch, oracle, alone): %s" % (len(bad), detail)
        assert s.count(2, 10 ** 11 + 1) == PI_1E11
