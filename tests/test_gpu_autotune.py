"""The autotuner times real candidates, rejects none that change results, and
caches its choice per (GPU, workload class)."""
import json

import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
pkg = pytest.importorskip("paper_2310_17746_amd")


def test_tune_and_cache(tmp_path, monkeypatch):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2310_17746_amd import autotune
    monkeypatch.setattr(autotune, "CACHE", str(tmp_path / "cache.json"))
    monkeypatch.setitem(autotune.GRIDS, "count",
                        [dict(segment_bytes=32768, block_threads=512, wg_per_cu=4, split_hits=32),
                         dict(segment_bytes=65536, block_threads=512, wg_per_cu=2, split_hits=64)])
    p = autotune.tuned("count")
    data = json.load(open(tmp_path / "cache.json"))
    (key,) = data.keys()
    assert key.endswith("|count") and "gfx950" in key
    assert len(data[key]["grid"]) == 3 and data[key]["ms"] <= data[key]["default_ms"]
    # the chosen parameters run and give the same answer
    with pkg.Sieve(0, p) as s:
        s.ensure_base_for(10 ** 10 + 1)
        assert s.count(2, 10 ** 10 + 1) == 455052511
    assert autotune.tuned("count") == p  # served from the cache
