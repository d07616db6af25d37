"""Autotuner for the sieve's launch parameters.

For a workload class it times a bounded grid of sieve_params on a
representative sample of that workload on the GPU at hand, keeps the fastest
setting, and caches the result in a JSON file keyed by (GPU architecture, CU
count, workload class).  The knobs are the paper's S (segment bytes per
tile) and t (threads per workgroup) of Fig. 4, plus workgroups per CU, the
tiles per strip, and the bucket-sieve threshold; each candidate is checked
to reproduce the counts of the default setting before it may win.

    from paper_2310_17746_amd import autotune
    params = autotune.tuned("batch")            # cached, or tuned now
    s = Sieve(0, params)
"""
from __future__ import annotations

import json
import os
import time

import numpy as np

from . import Sieve, load_library, workloads

CACHE = os.environ.get("SIEVE_AUTOTUNE_CACHE",
                       os.path.join(os.path.dirname(os.path.abspath(__file__)), "autotune_cache.json"))

# Candidate grids per workload class: (segment_bytes, block_threads, wg_per_cu, strip_tiles,
# bucket_threshold).  0 = automatic.  The default is one 1024-thread workgroup
# per CU with a 152 KiB tile; the other shapes trade the carried state for
# more waves per SIMD.
_SEGS = [(53248, 512, 3), (77824, 512, 2), (155648, 1024, 1), (131072, 1024, 1)]
GRIDS = {
    "count": [dict(segment_bytes=sg, block_threads=nt, wg_per_cu=w, strip_tiles=st)
              for sg, nt, w in _SEGS for st in (0, 4, 8)],
    "batch": [dict(segment_bytes=sg, block_threads=nt, wg_per_cu=w, bucket_threshold=bt)
              for sg, nt, w in _SEGS[:3] for bt in (0, 8 * sg)],
}


def _device_key() -> str:
    import torch
    p = torch.cuda.get_device_properties(0)
    arch = getattr(p, "gcnArchName", "unknown").split(":")[0]
    return "%s/%dcu" % (arch, p.multi_processor_count)


def _sample(kind: str):
    """A representative, bounded sample of the workload class."""
    if kind == "count":
        # the headline count itself (about 10 ms per call)
        return np.array([2], dtype=np.uint64), np.array([10 ** 11 + 1], dtype=np.uint64)
    if kind == "batch":
        # the whole 4096-range batch (about 10 ms per call): a subset has
        # fewer of the costly high single-tile ranges and ranks settings
        # differently
        lo, hi, _ = workloads.batch_ranges(0)
        return lo, hi
    raise ValueError("unknown workload class %r" % kind)


def _time(params: dict, lo, hi, reps: int = 5):
    with Sieve(0, params) as s:
        s.ensure_base_for(int(hi.max()))
        ref = s.count_batch(lo, hi)
        t0 = time.perf_counter()
        for _ in range(reps):
            s.count_batch(lo, hi)
        return (time.perf_counter() - t0) / reps, ref


# A candidate replaces the default only when it is faster by at least this
# fraction: run-to-run timing spread is about half a percent, and a tie
# would otherwise flip the chosen shape from run to run.
MARGIN = 0.01


def tune(kind: str, verbose: bool = False) -> dict:
    """Times the grid for `kind` and returns the fastest parameters (the
    default unless a candidate beats it by MARGIN)."""
    load_library()
    lo, hi = _sample(kind)
    base_t, want = _time({}, lo, hi)
    best, best_t = {}, base_t
    results = [({}, base_t)]
    for p in GRIDS[kind]:
        t, got = _time(p, lo, hi)
        if not np.array_equal(got, want):
            raise RuntimeError("autotune candidate %r changed the counts" % (p,))
        results.append((p, t))
        if verbose:
            print("autotune %s %r: %.3f ms" % (kind, p, t * 1e3), flush=True)
        if t < best_t:
            best, best_t = p, t
    if best_t > base_t * (1.0 - MARGIN):
        best, best_t = {}, base_t
    return {"params": best, "ms": best_t * 1e3, "default_ms": base_t * 1e3,
            "grid": [{"params": p, "ms": t * 1e3} for p, t in results]}


def tuned(kind: str, retune: bool = False, verbose: bool = False) -> dict:
    """Cached best parameters for `kind` on this GPU (tunes on a miss)."""
    key = "%s|%s" % (_device_key(), kind)
    cache = {}
    if os.path.exists(CACHE):
        with open(CACHE) as f:
            cache = json.load(f)
    if retune or key not in cache:
        cache[key] = tune(kind, verbose=verbose)
        tmp = CACHE + ".tmp%d" % os.getpid()
        with open(tmp, "w") as f:
            json.dump(cache, f, indent=1, sort_keys=True)
        os.replace(tmp, CACHE)
    return dict(cache[key]["params"])
