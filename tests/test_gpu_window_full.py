"""Full-size parity of the uint64 window list [10^12, 10^12 + 10^10), in the
launch configuration the benchmark times: default parameters, one list call
into a device buffer of list_bound entries, repeated into the same buffer.

The whole output (about 3.6e8 primes) is compared with the oracle: its
count, and the SHA-256 of every chunk of 2^24 primes against the oracle's
(tests/golden/window_1e12_1e10.txt).  A differing chunk is named, and its
values are then compared with the oracle's list of that chunk's span element
by element, which names the first differing index.  Sub-windows at the two
ends and across the boundaries of the default 52 KiB tiles are also compared
with a fresh oracle list directly.
"""
import random
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest

import oracle
from conftest import GOLDEN_CHUNK, assert_same_primes, chunk_digests, read_golden_results

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
pkg = pytest.importorskip("paper_2310_17746_amd")

LO, HI = 10 ** 12, 10 ** 12 + 10 ** 10
TILE_INTS = 24 * 53248


def _slice(out, n, a, b):
    """The listed values in [a, b), found by binary search on the device."""
    keys = torch.tensor([a, b], dtype=torch.int64, device=out.device)
    i, j = torch.searchsorted(out[:n], keys).tolist()
    return out[i:j].cpu().numpy().view(np.uint64)


def test_window_list_full_size():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    counts, chunks = read_golden_results("window_1e12_1e10.txt")
    want = chunks[0]
    s = pkg.Sieve(0, {})
    try:
        s.ensure_base_for(HI)
        cap = pkg.list_bound(LO, HI)
        out = torch.empty(cap, dtype=torch.int64, device="cuda")
        n = s.list(LO, HI, out=out, elem_bytes=8).numel()
        torch.cuda.synchronize()
        assert n == counts[0]

        host = out[:n].cpu().numpy().view(np.uint64)
        with ThreadPoolExecutor(16) as ex:
            got = [d for part in ex.map(lambda k: chunk_digests(host[k:k + GOLDEN_CHUNK]),
                                        range(0, n, GOLDEN_CHUNK)) for d in part]
        for k, (g, w) in enumerate(zip(got, want)):
            if g != w:
                # name the first differing element of this chunk
                ref = oracle.primes(w[0], w[1] + 1, elem_bytes=8)
                assert_same_primes(host[k * GOLDEN_CHUNK:k * GOLDEN_CHUNK + len(ref)], ref,
                                   "chunk %d of the window (elements from %d)" % (k, k * GOLDEN_CHUNK))
                raise AssertionError("chunk %d: got %s, oracle %s" % (k, g, w))
        assert len(got) == len(want)

        rng = random.Random(2310)
        windows = [(LO, LO + 10 ** 6), (HI - 10 ** 6, HI)]
        t0 = 192 * (LO // 192)
        for j in rng.sample(range(1, (HI - t0) // TILE_INTS), 8):
            b = t0 + j * TILE_INTS
            windows.append((b - 4096, b + 4096))
        for a, b in windows:
            assert_same_primes(_slice(out, n, a, b), oracle.primes(a, b, elem_bytes=8), "[%d, %d)" % (a, b))

        # the timed loop lists into the same buffer again: same result
        first = out[:n].clone()
        for _ in range(2):
            m = s.list(LO, HI, out=out, elem_bytes=8).numel()
            torch.cuda.synchronize()
            assert m == n
            assert torch.equal(out[:n], first)
    finally:
        s.close()
