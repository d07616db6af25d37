"""The autotuner's selection rule on the host (timings stubbed): the fastest
candidate wins only when it beats the default by the stated margin, and a
candidate that changes the counts is rejected."""
import numpy as np
import pytest

pkg = pytest.importorskip("paper_2310_17746_amd")
from paper_2310_17746_amd import autotune  # noqa: E402


def _stub(monkeypatch, times, counts=None):
    lo = np.array([2], dtype=np.uint64)
    hi = np.array([100], dtype=np.uint64)
    monkeypatch.setattr(autotune, "load_library", lambda: None)
    monkeypatch.setattr(autotune, "_sample", lambda kind: (lo, hi))
    grid = [dict(segment_bytes=8192 * (i + 1)) for i in range(len(times) - 1)]
    monkeypatch.setitem(autotune.GRIDS, "count", grid)
    seq = iter(zip(times, counts or [np.array([25])] * len(times)))
    monkeypatch.setattr(autotune, "_time", lambda p, lo, hi: next(seq))
    return grid


def test_tie_keeps_the_default(monkeypatch):
    _stub(monkeypatch, [10.0, 9.96, 9.97])  # 0.4% faster: within the margin
    r = autotune.tune("count")
    assert r["params"] == {} and r["ms"] == r["default_ms"] == 10.0e3


def test_clear_win_is_taken(monkeypatch):
    grid = _stub(monkeypatch, [10.0, 9.96, 9.7])  # 3% faster
    r = autotune.tune("count")
    assert r["params"] == grid[1] and abs(r["ms"] - 9.7e3) < 1e-6
    assert len(r["grid"]) == 3


def test_changed_counts_are_rejected(monkeypatch):
    _stub(monkeypatch, [10.0, 5.0], [np.array([25]), np.array([24])])
    with pytest.raises(RuntimeError):
        autotune.tune("count")
