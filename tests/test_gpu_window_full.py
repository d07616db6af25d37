"""Full-size parity of the uint64 window list [10^12, 10^12 + 10^10), in the
launch configuration the benchmark times: default parameters, one list call
into a device buffer of list_bound entries, repeated into the same buffer.

The oracle checks the count over the whole window and the listed values
element by element on sampled sub-windows: random ones, ones that straddle
the boundaries of the default 52 KiB tiles (24 * 53248 integers each), and
the two ends of the window.  Over the whole output the device checks what
holds at any size: strictly increasing, inside the window, every value
1 or 5 mod 6.
"""
import random

import numpy as np
import pytest

import oracle
from conftest import assert_same_primes

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
    s = pkg.Sieve(0, {})
    try:
        s.ensure_base_for(HI)
        cap = pkg.list_bound(LO, HI)
        out = torch.empty(cap, dtype=torch.int64, device="cuda")
        n = s.list(LO, HI, out=out, elem_bytes=8).numel()
        torch.cuda.synchronize()
        assert n == oracle.count(LO, HI)

        v = out[:n]
        assert bool((v[1:] > v[:-1]).all())
        assert int(v[0]) >= LO and int(v[-1]) < HI
        r = v % 6
        assert bool(((r == 1) | (r == 5)).all())
        del r

        rng = random.Random(2310)
        windows = [(LO, LO + 10 ** 6), (HI - 10 ** 6, HI)]
        for _ in range(16):
            a = rng.randrange(LO, HI - 10 ** 6)
            windows.append((a, a + 10 ** 6))
        t0 = 192 * (LO // 192)
        for j in rng.sample(range(1, (HI - t0) // TILE_INTS), 24):
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
