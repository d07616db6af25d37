import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

GOLDEN = os.path.join(ROOT, "tests", "golden")


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU")
    config.addinivalue_line("markers", "slow: long-running CPU test (minutes)")


def read_golden(name):
    """Rows of whitespace-separated fields from tests/golden/<name>, comments dropped."""
    rows = []
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.split("#", 1)[0].strip()
            if line:
                rows.append(line.split())
    return rows


@pytest.fixture(scope="session")
def pi_table():
    return {int(x): int(v) for x, v in read_golden("pi_values.txt")}


def first_mismatch(got, want):
    """Where two prime lists first differ: (index, got window, want window)
    around it, or None when they are equal.  Each window holds the values at
    index - 2 .. index + 2 that exist."""
    import numpy as np
    got = np.asarray(got)
    want = np.asarray(want)
    n = min(len(got), len(want))
    diff = np.nonzero(got[:n] != want[:n])[0]
    if len(diff):
        i = int(diff[0])
    elif len(got) != len(want):
        i = n
    else:
        return None
    lo = max(0, i - 2)
    return i, [int(v) for v in got[lo:i + 3]], [int(v) for v in want[lo:i + 3]]


def assert_same_primes(got, want, what=""):
    """Bit-exact list comparison that names the first differing index."""
    m = first_mismatch(got, want)
    assert m is None, "%s: lengths %d vs %d, first difference at index %d: got %s, want %s" % (
        what, len(got), len(want), m[0], m[1], m[2])

