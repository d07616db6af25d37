#!/usr/bin/env python3
"""Benchmark: sieved integers/s counting the primes of [2, 10^11] on one MI355X.

One step = one full pass of the sieve over the workload: a sieve_count call
on [2, 10^11 + 1) (tiling, presieve, Table 1 starts, LDS marking, edge masks,
popcount, per-range total), with the base primes <= isqrt(10^11) already
resident in HBM.  Prints one JSON line.  The launch shape (tile bytes,
threads, workgroups per CU, tiles per strip) is the autotuner's pick for this
workload, timed on it first, unless given on the command line.

The roofline entry ("bound": "lds") is for the dominant kernel (k_sieve):
its algorithmic LDS traffic (4 bytes per mark, read-modify-write of one
32-bit word, plus 8 bytes written per plane-word pair by the presieve and 8
bytes read back by the popcount) over its average duration, measured with
HIP events on the stream it runs on, against the nominal LDS bandwidth
derived from the unit counts (128 B/clk/CU * 256 CUs * 2.4 GHz).  The mark
count is exact: for every base prime p > 73 the number of m coprime to 30
with max(p^2, range base) <= m*p < range-span end.  Beside it: the measured
rate of the instruction itself (LDS probe, this run) and, from the committed
counter summary of the same kernel sources and launch shape, the LDS bytes
by counter, the HBM traffic and the VALU lane-ops against the derived VALU
peak (64 lanes/clk/CU * 256 CUs * 2.4 GHz).

The CPU baseline is the oracle (plain byte-per-integer segmented sieve, all
host threads) timed on a bounded slice of the same workload.

"extras" reports the other measured configurations in the same line:
* list_1e9: the sorted uint32 list of the primes in [2, 10^9]; the
  compaction phase (finalize + compaction kernels, HIP events) against HBM
  peak, with algorithmic bytes = 4 B per prime written + 8 B per bitmap word
  read.
* batch_4096: the 4096 seeded uneven ranges (half listed as uint64) in one
  batched call replaying a captured graph, against the same ranges as one
  plain call each; primes/s counts every prime counted or listed.  Its launch
  parameters come from the autotuner, run first on the same 4096 ranges
  (counted).
* serve_2000: 2000 seeded requests with Poisson arrivals at 0.8 x the
  saturated request rate (measured first with all requests at t = 0) and the
  count of [2, 10^12] submitted at t = 0; p50/p99 of completion - arrival.
* wide: windows past 2^64 (128-bit values): the count of
  [2^64, 2^64 + 10^10) and the list of [2^64, 2^64 + 10^9).
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PI_1E11 = 4118054813            # pi(10^11), standard published value
PI_1E12 = 37607912018           # pi(10^12), standard published value
LDS_PEAK_GBS = 128 * 256 * 2.4  # nominal LDS bandwidth, GB/s (B/clk/CU * CUs * GHz)
VALU_PEAK_LANE_OPS = 64 * 256 * 2.4e9  # int32 VALU lane-ops/s (lanes/clk/CU * CUs * Hz)


def small_primes(limit: int) -> np.ndarray:
    a = np.ones(limit + 1, dtype=bool)
    a[:2] = False
    for i in range(2, math.isqrt(limit) + 1):
        if a[i]:
            a[i * i::i] = False
    return np.nonzero(a)[0].astype(np.int64)


def coprime6_upto(n: np.ndarray) -> np.ndarray:
    """#{1 <= m <= n : gcd(m, 6) = 1}, elementwise, n >= 0."""
    q, s = np.divmod(n, 6)
    return 2 * q + (s >= 1) + (s >= 5)


_C30 = np.array([sum(1 for m in range(1, r + 1) if math.gcd(m, 30) == 1) for r in range(30)])


def coprime30_upto(n: np.ndarray) -> np.ndarray:
    """#{1 <= m <= n : gcd(m, 30) = 1}, elementwise, n >= 0."""
    q, s = np.divmod(n, 30)
    return 8 * q + _C30[s]


def lds_work(lo: int, hi: int, segment_bytes: int) -> tuple[int, int]:
    """(marks, plane words) the sieve kernel performs on [lo, hi).

    Primes 5..73 are presieved; every other base prime p marks p*m for the
    cofactors m coprime to 30 (multiples of 2, 3 are outside the wheel and
    multiples of 5 are already cleared by the presieve)."""
    base = lo - lo % 6
    n1 = (hi - base - 1 + 5) // 6
    words = (n1 + 31) // 32
    end = base + 192 * words
    p = small_primes(math.isqrt(hi - 1))
    p = p[p > 73]                                  # 5..73 are presieved by patterns
    # per tile the start is max(p^2, tile base); the sum over the tiles is the
    # sum over the whole span with the p^2 clamp, since tiles are contiguous
    # (the tile size only sets where they meet: segment_bytes does not change
    # the total)
    del segment_bytes
    start = np.maximum(p * p, base)
    m_lo = -(-start // p)
    m_hi = (end - 1) // p
    ok = m_hi >= m_lo
    marks = int(np.sum(np.where(ok, coprime30_upto(m_hi) - coprime30_upto(m_lo - 1), 0)))
    return marks, int(words)


KERNEL_SOURCES = ("paper_2310_17746_amd/csrc/kernels.hip", "paper_2310_17746_amd/csrc/wheel.h",
                  "paper_2310_17746_amd/csrc/sieve_internal.h")


def kernel_sources_sha() -> str:
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(params):
    """Counter figures per k_sieve dispatch from the committed summary: the
    entry taken with the same launch shape, if the summary was taken on the
    current kernel sources (else None)."""
    path = os.path.join(ROOT, "profiles", "k_sieve_pi1e11_traffic.json")
    try:
        with open(path) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if t.get("kernel_sources_sha256") != kernel_sources_sha():
        return None
    shape = ("segment_bytes", "block_threads", "wg_per_cu", "strip_tiles")
    for e in t.get("entries", []):
        if all(e.get("params", {}).get(k) == params.get(k) for k in shape):
            return e
    return None


def bench_list(pkg, torch, params, steps=5):
    """Sorted uint32 list of the primes in [2, 10^9]."""
    lo, hi = 2, 10 ** 9 + 1
    s = pkg.Sieve(0, params)
    s.ensure_base_for(hi)
    out = torch.empty(pkg.list_bound(lo, hi), dtype=torch.int32, device="cuda")
    n = s.list(lo, hi, out=out, elem_bytes=4).numel()
    torch.cuda.synchronize()
    s.set_timing(True)
    t0 = time.perf_counter()
    for _ in range(steps):
        s.list(lo, hi, out=out, elem_bytes=4)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    sieve_ms, post_ms, jobs = s.timing()
    s.close()
    words = ((hi - lo + 5) // 6 + 31) // 32
    post = post_ms / jobs
    nbytes = 4 * n + 8 * words
    gbs = nbytes / (post * 1e-3) / 1e9
    return {"workload": "sorted uint32 list of the primes in [2, 10^9]", "primes": n,
            "ms_per_call": round(dt * 1e3, 3), "ints_per_s": round((hi - lo) / dt, 1),
            "primes_per_s": round(n / dt, 1), "sieve_kernel_ms": round(sieve_ms / jobs, 4),
            "compaction_ms": round(post, 4),
            "compaction_roofline": {"bound": "hbm", "achieved": round(gbs, 1), "peak": 8000.0,
                                    "unit": "GB/s", "frac": round(gbs / 8000.0, 4),
                                    "algorithmic_bytes": nbytes}}


def bench_list_window(pkg, torch, params, steps=3):
    """Sorted uint64 list of the primes in the window [10^12, 10^12 + 10^10)."""
    lo, hi = 10 ** 12, 10 ** 12 + 10 ** 10
    s = pkg.Sieve(0, params)
    s.ensure_base_for(hi)
    out = torch.empty(pkg.list_bound(lo, hi), dtype=torch.int64, device="cuda")
    n = s.list(lo, hi, out=out, elem_bytes=8).numel()
    torch.cuda.synchronize()
    s.set_timing(True)
    t0 = time.perf_counter()
    for _ in range(steps):
        s.list(lo, hi, out=out, elem_bytes=8)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    sieve_ms, post_ms, jobs = s.timing()
    s.close()
    words = ((hi - lo + 5) // 6 + 31) // 32
    post = post_ms / jobs
    nbytes = 8 * n + 8 * words
    gbs = nbytes / (post * 1e-3) / 1e9
    # measured write ceiling: a plain device fill of the same output bytes
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    out[:n].fill_(7)
    e0.record()
    for _ in range(5):
        out[:n].fill_(7)
    e1.record()
    torch.cuda.synchronize()
    fill_gbs = 8 * n / (e0.elapsed_time(e1) / 5 * 1e-3) / 1e9
    return {"workload": "sorted uint64 list of the primes in [10^12, 10^12 + 10^10)", "primes": n,
            "ms_per_call": round(dt * 1e3, 3), "primes_per_s": round(n / dt, 1),
            "sieve_kernel_ms": round(sieve_ms / jobs, 4), "compaction_ms": round(post, 4),
            "compaction_roofline": {"bound": "hbm", "achieved": round(gbs, 1), "peak": 8000.0,
                                    "unit": "GB/s", "frac": round(gbs / 8000.0, 4),
                                    "algorithmic_bytes": nbytes, "fill_GB_per_s": round(fill_gbs, 1),
                                    "frac_of_fill": round(gbs / fill_gbs, 4)}}


def bench_cold(pkg, torch, params, hi=10 ** 11 + 1):
    """The headline count from a fresh context: creation, base primes, first count."""
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s = pkg.Sieve(0, params)
    t1 = time.perf_counter()
    s.ensure_base_for(hi)
    t2 = time.perf_counter()
    c = s.count(2, hi)
    t3 = time.perf_counter()
    c2 = s.count(2, hi)
    t4 = time.perf_counter()
    s.close()
    return {"workload": "count of [2, 10^11 + 1) from a fresh context", "count_ok": c == c2 == 4118054813,
            "create_ms": round((t1 - t0) * 1e3, 3), "base_primes_ms": round((t2 - t1) * 1e3, 3),
            "first_count_ms": round((t3 - t2) * 1e3, 3), "second_count_ms": round((t4 - t3) * 1e3, 3),
            "cold_total_ms": round((t3 - t0) * 1e3, 3)}


def bench_batch(pkg, torch, params, workloads, steps=3):
    """4096 seeded uneven ranges (seed 0, lo up to 10^15), half listed as uint64."""
    lo, hi, mode = workloads.batch_ranges(0)
    s = pkg.Sieve(0, dict(params, use_graph=1))
    s.ensure_base_for(int(hi.max()))
    cap = np.array([pkg.list_bound(int(a), int(b)) if m else 0 for a, b, m in zip(lo, hi, mode)],
                   dtype=np.uint64)
    off = np.concatenate([[0], np.cumsum(cap)[:-1]]).astype(np.uint64)
    out = torch.empty(int(cap.sum()) + 1, dtype=torch.int64, device="cuda")
    counts, status = s.list_batch(lo, hi, mode, out, off, cap, elem_bytes=8)  # warm-up + capture
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        counts, status = s.list_batch(lo, hi, mode, out, off, cap, elem_bytes=8)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    # the same ranges as one plain call each
    t1 = time.perf_counter()
    for a, b, m, o, c in zip(lo.tolist(), hi.tolist(), mode.tolist(), off.tolist(), cap.tolist()):
        if m:
            s.list(a, b, out=out[o:o + max(c, 1)], elem_bytes=8)
        else:
            s.count(a, b)
    torch.cuda.synchronize()
    dt_single = time.perf_counter() - t1
    s.close()
    # kernel time per phase of one batch, by HIP events on the stream the
    # kernels run on (events need the launches outside a graph)
    s = pkg.Sieve(0, dict(params, use_graph=0))
    s.ensure_base_for(int(hi.max()))
    s.list_batch(lo, hi, mode, out, off, cap, elem_bytes=8)
    torch.cuda.synchronize()
    s.set_timing(True)
    s.list_batch(lo, hi, mode, out, off, cap, elem_bytes=8)
    torch.cuda.synchronize()
    sieve_ms, post_ms, bucket_ms, jobs = s.timing_all()
    # the same ranges one call each, device time only (the same events,
    # summed over the 4096 jobs): the batching gain without host overhead
    s.set_timing(True)
    for a, b, m, o, c in zip(lo.tolist(), hi.tolist(), mode.tolist(), off.tolist(), cap.tolist()):
        if m:
            s.list(a, b, out=out[o:o + max(c, 1)], elem_bytes=8)
        else:
            s.count(a, b)
    torch.cuda.synchronize()
    r_sieve, r_post, r_bucket, r_jobs = s.timing_all()
    s.close()
    dev_batch = sieve_ms + post_ms + bucket_ms
    dev_single = r_sieve + r_post + r_bucket
    ints = int((hi - lo).sum())
    primes = int(counts.sum())
    return {"workload": "4096 ranges (seed 0): lo log-uniform [1e6, 1e15], length log-uniform "
                        "[1e3, 1e8], half listed as uint64", "ok": bool(np.all(status == 0)),
            "ints": ints, "primes": primes, "listed": int(counts[mode == 1].sum()),
            "ms_per_batch": round(dt * 1e3, 3), "ints_per_s": round(ints / dt, 1),
            "primes_per_s": round(primes / dt, 1),
            "per_range_ms": round(dt_single * 1e3, 3),
            "batched_vs_per_range": round(dt_single / dt, 3),
            "device_ms": {"batched": round(dev_batch, 3), "per_range_sum": round(dev_single, 3),
                          "per_range_jobs": r_jobs, "batched_vs_per_range": round(dev_single / dev_batch, 3)},
            "phases_ms": {"sieve": round(sieve_ms, 3), "bucket_fill": round(bucket_ms, 3),
                          "scan_and_compaction": round(post_ms, 3), "jobs": jobs}}


def bench_stream(pkg, torch, params):
    """Incremental generation and streaming to host memory."""
    s = pkg.Sieve(0, params)
    # Generator: 2^24 primes per call from 10^12 (device output, uint64).
    g = s.generator(10 ** 12, 8)
    out = torch.empty(1 << 24, dtype=torch.int64, device="cuda")
    g.next(1 << 24, out=out)  # warm-up: base primes, staging buffer
    torch.cuda.synchronize()
    calls = 8
    t0 = time.perf_counter()
    for _ in range(calls):
        g.next(1 << 24, out=out)
    torch.cuda.synchronize()
    dt_gen = (time.perf_counter() - t0) / calls
    pos = g.position
    g.close()
    # Host stream: the uint64 list of [10^12, 10^12 + 10^10) into pinned host memory.
    lo, hi = 10 ** 12, 10 ** 12 + 10 ** 10
    s.ensure_base_for(hi)
    host = torch.empty(pkg.list_bound(lo, hi), dtype=torch.int64, pin_memory=True)
    s.list_host(lo, lo + 10 ** 8, elem_bytes=8, out=host)  # warm-up: pipeline buffers
    t1 = time.perf_counter()
    n = len(s.list_host(lo, hi, elem_bytes=8, out=host))
    dt_host = time.perf_counter() - t1
    s.close()
    return {"generator": {"workload": "sieve_gen_next of 2^24 uint64 primes per call from 10^12",
                          "ms_per_call": round(dt_gen * 1e3, 3),
                          "primes_per_s": round((1 << 24) / dt_gen, 1), "position_after": pos},
            "list_host": {"workload": "uint64 list of [10^12, 10^12 + 10^10) streamed to pinned host memory",
                          "primes": n, "ms": round(dt_host * 1e3, 3), "primes_per_s": round(n / dt_host, 1),
                          "host_GB_per_s": round(8 * n / dt_host / 1e9, 2)}}


def bench_serve(pkg, workloads):
    """2000 seeded requests (seed 1) on a Poisson stream, with the [2, 10^12] count job beside it."""
    lo, hi, mode, gaps = workloads.serving_requests(1)
    long_lo, long_hi = workloads.LONG_JOB
    s = pkg.Sieve(0)
    s.ensure_base_for(max(int(hi.max()), long_hi))
    n = len(lo)

    def run(arrivals_ns, **sp):
        with pkg.Server(s, out_budget_bytes=64 << 30, elem_bytes=8, **sp) as srv:
            t0 = srv.now_ns() + 2_000_000
            srv.submit(long_lo, long_hi, 0, n, at_ns=t0)
            for i in range(n):
                srv.submit(int(lo[i]), int(hi[i]), int(mode[i]), i, at_ns=t0 + int(arrivals_ns[i]))
            done = {}
            t_end = time.time() + 300
            while len(done) < n + 1:
                if time.time() > t_end:
                    raise RuntimeError("serving run did not finish")
                for c in srv.poll(4096, wait_ms=20):
                    done[c["tag"]] = c
                    if c["mode"] == 1 and c["status"] == 0:
                        srv.release(c["tag"])
            st = srv.stats()
        return done, st, t0

    # saturated rate: every request arrives at once (after one such run that
    # grows the context's job scratch and bucket pool to the mix's size)
    run(np.zeros(n))
    done, st, t0 = run(np.zeros(n))
    t_sat = max(done[i]["t_done_ns"] for i in range(n)) - t0
    mu = n / (t_sat * 1e-9)
    lam = 0.8 * mu
    arrivals = np.cumsum(gaps) / lam * 1e9
    done, st, t0 = run(arrivals)
    lat = np.array([(done[i]["t_done_ns"] - done[i]["t_arrival_ns"]) * 1e-6 for i in range(n)])
    # the same saturated run with step k + 1 enqueued while step k runs
    done_o, st_o, t0_o = run(np.zeros(n), overlap=1)
    mu_o = n / ((max(done_o[i]["t_done_ns"] for i in range(n)) - t0_o) * 1e-9)
    # every request finished, and the long job's count is pi(10^12)
    ok = all(done[i]["status"] == 0 for i in range(n + 1)) and int(done[n]["count"]) == PI_1E12
    span = (max(c["t_done_ns"] for c in done.values()) - t0) * 1e-9
    ints = int((hi - lo).sum())
    s.close()
    return {"workload": "2000 requests (seed 1): lo log-uniform [1e6, 1e14], length log-uniform "
                        "[1e4, 1e9], 30% listed as uint64, Poisson arrivals; plus the count of "
                        "[2, 1e12] at t = 0", "ok": ok,
            "saturated_req_per_s": round(mu, 1), "lambda_req_per_s": round(lam, 1),
            "saturated_req_per_s_overlap": round(mu_o, 1),
            "p50_ms": round(float(np.percentile(lat, 50)), 3),
            "p99_ms": round(float(np.percentile(lat, 99)), 3),
            "mean_ms": round(float(lat.mean()), 3),
            "long_job_ms": round((done[n]["t_done_ns"] - done[n]["t_arrival_ns"]) * 1e-6, 3),
            "long_job_count": int(done[n]["count"]),
            "ints_per_s": round((ints + long_hi - long_lo) / span, 1),
            "req_per_s": round(n / span, 1),
            # device time of the steps' jobs over the span from the first
            # arrival to the last completion
            "utilization": round(st["busy_ns"] / max(span * 1e9, 1), 4),
            "steps": st["steps"], "overlap_steps": st["overlap_steps"],
            # steps that ran the bucket sieve; pieces that resumed their
            # request's walks from the device-resident state, and its memory
            "bucket_steps": st["bucket_steps"], "resumed_walks": st["resumed_walks"],
            "walk_state_bytes": st["walk_bytes"]}


def bench_walks(pkg):
    """Requests cut into many pieces that take the bucket sieve: 24 counts of
    10^8 integers from lo log-uniform in [10^13, 10^14] (seed 3), two-tile
    pieces.  Device time of the serving steps with each request's bucket walk
    state kept on the device between pieces, against every piece restarting
    its walks; the counts must agree."""
    rng = np.random.default_rng(3)
    n = 24
    lo = np.floor(10 ** rng.uniform(13, 14, n)).astype(np.uint64)
    hi = lo + np.uint64(10 ** 8)
    s = pkg.Sieve(0)
    s.ensure_base_for(int(hi.max()))
    res = {}
    for restart in (0, 1, 0, 1):  # the second run of each mode is kept
        with pkg.Server(s, step_tiles=64, quantum_tiles=2, restart_walks=restart) as srv:
            t0 = time.perf_counter()
            for i in range(n):
                srv.submit(int(lo[i]), int(hi[i]), 0, i)
            done = {}
            t_end = time.time() + 120
            while len(done) < n:
                if time.time() > t_end:
                    raise RuntimeError("walk run did not finish")
                for c in srv.poll(64, wait_ms=20):
                    done[c["tag"]] = c
            wall = time.perf_counter() - t0
            st = srv.stats()
        res[restart] = {"busy_ms": round(st["busy_ns"] * 1e-6, 3), "wall_ms": round(wall * 1e3, 3),
                        "steps": st["steps"], "busy_ms_per_step": round(st["busy_ns"] * 1e-6 / max(st["steps"], 1), 4),
                        "bucket_steps": st["bucket_steps"],
                        "resumed_walks": st["resumed_walks"], "walk_state_bytes": st["walk_bytes"],
                        "counts": [int(done[i]["count"]) for i in range(n)],
                        "ok": all(done[i]["status"] == 0 for i in range(n))}
    s.close()
    ok = res[0]["ok"] and res[1]["ok"] and res[0]["counts"] == res[1]["counts"]
    for r in res.values():
        del r["counts"], r["ok"]
    return {"workload": "24 counts of 10^8 integers from lo log-uniform [1e13, 1e14] (seed 3), served in "
                        "two-tile pieces", "ok": ok, "resident_walks": res[0], "restarted_walks": res[1],
            # (wall time includes the new server's allocation of the walk buffers)
            "busy_per_step_ratio_resident_over_restarted":
                round(res[0]["busy_ms_per_step"] / max(res[1]["busy_ms_per_step"], 1e-9), 3)}


def bench_wide(pkg, torch, params, steps=3):
    """Windows past 2^64 (128-bit values): the count of [2^64, 2^64 + 10^10)
    and the list of [2^64, 2^64 + 10^9), with the base primes below 2^32
    resident and the extension list reaching isqrt(2^64 + 10^10)."""
    T64 = 1 << 64
    s = pkg.Sieve(0, params)
    t0 = time.perf_counter()
    s.base_primes((1 << 32) - 1)
    clo, chi = T64, T64 + 10 ** 10
    s.ensure_base_wide_for(chi)
    base_s = time.perf_counter() - t0
    n = s.count_wide(clo, chi)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for _ in range(steps):
        s.count_wide(clo, chi)
    dt_c = (time.perf_counter() - t1) / steps
    llo, lhi = T64, T64 + 10 ** 9
    out = torch.empty((pkg.list_bound_wide(llo, lhi), 2), dtype=torch.int64, device="cuda")
    m = s.list_wide(llo, lhi, out=out).shape[0]
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    for _ in range(steps):
        s.list_wide(llo, lhi, out=out)
    dt_l = (time.perf_counter() - t2) / steps
    s.close()
    return {"workload": "count of [2^64, 2^64 + 10^10) and 128-bit list of [2^64, 2^64 + 10^9)",
            "count": n, "count_ms": round(dt_c * 1e3, 3), "count_ints_per_s": round((chi - clo) / dt_c, 1),
            "listed": m, "list_ms": round(dt_l * 1e3, 3), "list_ints_per_s": round((lhi - llo) / dt_l, 1),
            "base_primes_s": round(base_s, 2)}


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def oracle_other_workloads(oracle, threads):
    """The oracle on bounded samples of configs 1, 2, 4 and 5 and of the
    window list, on `threads` threads and (on a smaller sample) on one."""
    from paper_2310_17746_amd import workloads as wl
    blo, bhi, _ = wl.batch_ranges(0)
    bsel = np.random.default_rng(3).choice(len(blo), 64, replace=False)
    slo, shi, smode, _ = wl.serving_requests(1)
    short = np.nonzero(shi - slo <= 10 ** 8)[0]
    ssel = np.random.default_rng(4).choice(short, 32, replace=False)

    def batch(sel, th):
        return sum(oracle.count(int(blo[i]), int(bhi[i]), threads=th) for i in sel)

    def serve(sel, th):
        n = 0
        for i in sel:
            if smode[i]:
                n += len(oracle.primes(int(slo[i]), int(shi[i]), elem_bytes=8, threads=th))
            else:
                n += oracle.count(int(slo[i]), int(shi[i]), threads=th)
        return n

    def lst(lo, hi, eb):
        return lambda th: len(oracle.primes(lo, hi, elem_bytes=eb, threads=th))

    # name: (all-threads sample, its integers, its call), (one-thread sample, integers, call)
    cases = {
        "list_1e7": (("[2, 10^7 + 1) listed as uint32", 10 ** 7 - 1, lst(2, 10 ** 7 + 1, 4)),
                         ("the same", 10 ** 7 - 1, lst(2, 10 ** 7 + 1, 4))),
        "list_1e9": (("[2, 10^9 + 1) listed as uint32", 10 ** 9 - 1, lst(2, 10 ** 9 + 1, 4)),
                         ("[2, 10^8 + 1) listed as uint32", 10 ** 8 - 1, lst(2, 10 ** 8 + 1, 4))),
        "list_window_sample": (("[10^12, 10^12 + 10^8) listed as uint64", 10 ** 8,
                                lst(10 ** 12, 10 ** 12 + 10 ** 8, 8)),
                               ("[10^12, 10^12 + 2 10^7) listed as uint64", 2 * 10 ** 7,
                                lst(10 ** 12, 10 ** 12 + 2 * 10 ** 7, 8))),
        "batch_sample": (("64 of the 4096 seeded batch ranges (seed 0), counted", int((bhi[bsel] - blo[bsel]).sum()),
                          lambda th: batch(bsel, th)),
                         ("16 of those 64", int((bhi[bsel[:16]] - blo[bsel[:16]]).sum()),
                          lambda th: batch(bsel[:16], th))),
        "serve_sample": (("32 of the 2000 seeded serving requests (seed 1) of at most 10^8 integers (counted or listed as uint64)",
                          int((shi[ssel] - slo[ssel]).sum()), lambda th: serve(ssel, th)),
                         ("8 of those 32", int((shi[ssel[:8]] - slo[ssel[:8]]).sum()),
                          lambda th: serve(ssel[:8], th))),
    }
    out = {}
    for name, (full, small) in cases.items():
        r = {}
        for tag, th, (sample, ints, fn) in (("all_threads", threads, full), ("one_thread", 1, small)):
            t0 = time.perf_counter()
            primes = fn(th)
            dt = time.perf_counter() - t0
            r[tag] = {"sample": sample, "ms": round(dt * 1e3, 1), "ints_per_s": round(ints / dt, 1),
                      "primes_per_s": round(primes / dt, 1)}
        out[name] = r
    return out


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--hi", type=int, default=10 ** 11 + 1)
    ap.add_argument("--segment-bytes", type=int, default=0)
    ap.add_argument("--block-threads", type=int, default=0)
    ap.add_argument("--wg-per-cu", type=int, default=0)
    ap.add_argument("--split-hits", type=int, default=0)
    ap.add_argument("--presieve-groups", type=int, default=0)
    ap.add_argument("--strip-tiles", type=int, default=0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true", help="headline count only")
    ap.add_argument("--cpu-sample", type=int, default=10 ** 11,
                    help="integers of the oracle's timed slice (the top of the range)")
    ap.add_argument("--extra", default="",
                    choices=["", "list_1e9", "list_window", "batch_4096", "serve_2000", "walks", "wide"],
                    help="run only this extra workload and print its JSON (for profiling)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="BYTES",
                    help="only run a plain device-to-device copy of BYTES (5 times), the reference "
                         "for scaling the FETCH_SIZE / WRITE_SIZE counters")
    args = ap.parse_args()

    if args.copy_calibration:
        import torch
        a = torch.ones(args.copy_calibration // 4, dtype=torch.int32, device="cuda")
        b = torch.empty_like(a)
        for _ in range(5):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes": a.numel() * 4, "copies": 5}), flush=True)
        return 0

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the library runs on a single GPU and has no "
              "multi-GPU path; run with --gpus 1", file=sys.stderr)
        return 2

    import torch
    import paper_2310_17746_amd as pkg

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        return 2
    lo, hi = 2, args.hi
    params = {k: v for k, v in dict(segment_bytes=args.segment_bytes, block_threads=args.block_threads,
                                     wg_per_cu=args.wg_per_cu, split_hits=args.split_hits,
                                     presieve_groups=args.presieve_groups,
                                     strip_tiles=args.strip_tiles).items() if v}
    if args.extra:
        from paper_2310_17746_amd import workloads
        fn = {"list_1e9": lambda: bench_list(pkg, torch, params),
              "list_window": lambda: bench_list_window(pkg, torch, params),
              "batch_4096": lambda: bench_batch(pkg, torch, params, workloads),
              "serve_2000": lambda: bench_serve(pkg, workloads),
              "walks": lambda: bench_walks(pkg),
              "wide": lambda: bench_wide(pkg, torch, params)}[args.extra]
        print(json.dumps({"extra": args.extra, **fn()}), flush=True)
        return 0
    # Launch shape of the headline count: the autotuner's pick for this very
    # workload (timed on it, counts checked against the default's), unless
    # the shape is given on the command line.
    hparams, tuned_count = dict(params), None
    if not any(k in params for k in ("segment_bytes", "block_threads", "wg_per_cu", "strip_tiles")):
        from paper_2310_17746_amd import autotune
        print("bench: autotune count", file=sys.stderr, flush=True)
        tuned_count = autotune.tune("count")
        hparams.update(tuned_count["params"])
    s = pkg.Sieve(0, hparams)
    s.ensure_base_for(hi)                     # base primes resident before timing
    prm = s.params.as_dict()
    print("bench: count [%d, %d) params %s" % (lo, hi, prm), file=sys.stderr, flush=True)

    for _ in range(args.warmup):
        c = s.count(lo, hi)
    torch.cuda.synchronize()
    s.set_timing(True)
    t0 = time.perf_counter()
    for _ in range(args.steps):
        c = s.count(lo, hi)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    sieve_ms, post_ms, jobs = s.timing()
    s.set_timing(False)
    dt = t1 - t0
    ints = hi - lo
    value = ints * args.steps / dt
    count_ok = (c == PI_1E11) if hi == 10 ** 11 + 1 else None

    marks, words = lds_work(lo, hi, prm["segment_bytes"])
    lds_bytes = 4 * marks + 16 * words
    k_ms = sieve_ms / max(jobs, 1)
    achieved = lds_bytes / (k_ms * 1e-3) / 1e9
    tr = measured_traffic(prm) if hi == 10 ** 11 + 1 else None
    # bound "lds": the marks are 32-bit LDS read-modify-writes, and achieved /
    # peak is an LDS bandwidth fraction against the nominal LDS rate derived
    # from the unit counts (128 B/clk/CU x 256 CUs x 2.4 GHz)
    roof = {"bound": "lds", "resource": "LDS read-modify-write of 32-bit words (ds_or_b32)",
            "achieved": round(achieved, 1), "peak": round(LDS_PEAK_GBS, 1), "unit": "GB/s",
            "frac": round(achieved / LDS_PEAK_GBS, 4),
            "peak_source": "derived: 128 B/clk/CU x 256 CUs x 2.4 GHz",
            "traffic": (tr["fetch_bytes"] + tr["write_bytes"]) if tr else None,
            "kernel": "k_sieve", "kernel_ms": round(k_ms, 4), "marks": marks,
            "algorithmic_bytes": lds_bytes}
    # Measured peak of the instruction the marks use (32-bit LDS OR), from the
    # library's LDS probe in this run: conflict-free and random-word patterns.
    probe = {}
    for mode in ("or_linear", "or_random"):
        ops, _ = pkg.probe_lds(mode, iters=2048, wg_per_cu=2)
        probe[mode] = ops * 4 / 1e9  # GB/s of 4-byte read-modify-writes
    roof["instr_peak"] = {"instruction": "ds_or_b32", "unit": "GB/s",
                          "conflict_free": round(probe["or_linear"], 1),
                          "frac_conflict_free": round(achieved / probe["or_linear"], 4),
                          "random_words": round(probe["or_random"], 1),
                          "frac_random_words": round(achieved / probe["or_random"], 4)}
    if tr:
        # from the committed counter summary of the same kernel sources and
        # launch shape, over this run's kernel time
        cb = tr["lds_counter_bytes"] / (k_ms * 1e-3) / 1e9
        roof["lds_counter"] = {"bytes": int(tr["lds_counter_bytes"]), "GB_per_s": round(cb, 1),
                               "frac_conflict_free": round(cb / probe["or_linear"], 4),
                               "frac_nominal": round(cb / roof["peak"], 4),
                               "bank_conflict_share": round(tr["lds_bank_conflict"], 4)}
        lane_ops = tr["sq_insts_valu"] * 64 / (k_ms * 1e-3)
        roof["alu"] = {"achieved": round(lane_ops, 1), "peak": VALU_PEAK_LANE_OPS, "unit": "VALU lane-ops/s",
                       "frac": round(lane_ops / VALU_PEAK_LANE_OPS, 4),
                       "peak_source": "derived: 64 lanes/clk/CU (4 SIMD x 16) x 256 CUs x 2.4 GHz",
                       "valu_per_mark": round(tr["sq_insts_valu"] * 64 / marks, 2)}

    s.close()
    extras = None
    if not args.no_extras:
        from paper_2310_17746_amd import workloads
        extras = {}
        from paper_2310_17746_amd import autotune
        print("bench: autotune batch", file=sys.stderr, flush=True)
        tuned = autotune.tune("batch")
        bparams = dict(params, **tuned["params"])
        for name, fn in (("cold", lambda: bench_cold(pkg, torch, params)),
                         ("list_1e9", lambda: bench_list(pkg, torch, params)),
                         ("list_window", lambda: bench_list_window(pkg, torch, params)),
                         ("batch_4096", lambda: bench_batch(pkg, torch, bparams, workloads)),
                         ("stream", lambda: bench_stream(pkg, torch, params)),
                         ("serve_2000", lambda: bench_serve(pkg, workloads)),
                         ("walks", lambda: bench_walks(pkg)),
                         ("wide", lambda: bench_wide(pkg, torch, params))):
            print("bench: %s" % name, file=sys.stderr, flush=True)
            extras[name] = fn()
        extras["batch_4096"]["autotune"] = {"chosen": tuned["params"], "sample_ms": round(tuned["ms"], 3),
                                            "default_sample_ms": round(tuned["default_ms"], 3),
                                            "candidates": len(tuned["grid"])}

    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        th = oracle.default_threads()
        a = max(lo, hi - args.cpu_sample)
        t2 = time.perf_counter()
        oc = oracle.count(a, hi, threads=th)
        t3 = time.perf_counter()
        cpu = {"value": round((hi - a) / (t3 - t2), 1), "unit": "ints/s", "cores": th, "kind": "oracle",
               "sample": "oracle count of [%d, %d) (%d integers, the top of the workload): %d primes in %.2f s"
                         % (a, hi, hi - a, oc, t3 - t2)}
        # the oracle on the other workloads (context for the extras; bounded
        # samples), on all threads and on one
        cpu["cpu_model"] = cpu_model()
        cpu["other_workloads"] = oracle_other_workloads(oracle, th)
        # the same oracle on one thread, over the top 10^9 integers of the workload
        a1 = max(lo, hi - 10 ** 9)
        t4 = time.perf_counter()
        oracle.count(a1, hi, threads=1)
        t5 = time.perf_counter()
        cpu["one_thread"] = {"value": round((hi - a1) / (t5 - t4), 1), "unit": "ints/s",
                             "sample": "oracle count of [%d, %d) on 1 thread" % (a1, hi)}

    line = {
        "metric": "sieved integers/s at pi(1e11) count",
        "value": round(value, 1),
        "unit": "ints/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(dt / args.steps * 1e3, 4),
        "higher_is_better": True,
        "scaling": "strong",
        "vs_baseline": None,
        "dtype": "u64",
        "data": "synthetic",
        "config": {"workload": "count the primes in [2, 10^11] (half-open [2, 10^11 + 1))",
                   "lo": lo, "hi": hi, "base_prime_limit": math.isqrt(hi - 1), **prm,
                   "shape_autotune": None if tuned_count is None else {
                       "chosen": tuned_count["params"], "ms": round(tuned_count["ms"], 3),
                       "default_ms": round(tuned_count["default_ms"], 3),
                       "candidates": len(tuned_count["grid"])}},
        "count": int(c),
        "count_ok": count_ok,
        "roofline": roof,
        "cpu_baseline": cpu,
        "extras": extras,
    }
    print(json.dumps(line), flush=True)
    return 0 if count_ok is not False else 1


if __name__ == "__main__":
    sys.exit(main())
