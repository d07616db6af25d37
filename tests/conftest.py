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



# Oracle results of the full-size workloads (tests/golden/make_golden.py):
# C rows give counts, L rows the SHA-256 digests of each list, per chunk of
# GOLDEN_CHUNK elements.
GOLDEN_CHUNK = 1 << 24


def read_golden_results(name):
    """(counts, chunks) from a results file: counts[i] = int and, for listed
    entries, chunks[i] = [(first, last, n, digest), ...] in chunk order."""
    counts, chunks = {}, {}
    for row in read_golden(name):
        if row[0] == "C":
            counts[int(row[1])] = int(row[2])
        elif row[0] == "L":
            lst = chunks.setdefault(int(row[1]), [])
            assert int(row[2]) == len(lst), "chunk rows out of order in %s" % name
            lst.append((int(row[3]), int(row[4]), int(row[5]), row[6]))
    return counts, chunks


def chunk_digests(v):
    """[(first, last, n, digest)] of a uint64 list, as the golden files hold them."""
    import hashlib

    import numpy as np
    v = np.ascontiguousarray(v, dtype="<u8")
    out = []
    for s in range(0, len(v), GOLDEN_CHUNK):
        c = v[s:s + GOLDEN_CHUNK]
        out.append((int(c[0]), int(c[-1]), len(c), hashlib.sha256(c.tobytes()).hexdigest()[:32]))
    return out


def golden_mismatch(got, want):
    """None when the digests agree, else a message naming the first differing
    chunk, its element offset and the value span the oracle gives for it."""
    if got == want:
        return None
    for k in range(max(len(got), len(want))):
        g = got[k] if k < len(got) else None
        w = want[k] if k < len(want) else None
        if g != w:
            return ("chunk %d (elements from %d): got %s, oracle %s"
                    % (k, k * GOLDEN_CHUNK, g, w))
    return "chunk lists differ"
