"""Oracle for the segmented wheel sieve -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The product path (the HIP library and
its Python binding) never imports it, and the two share no code.

Contents
--------
* ``count`` / ``primes``: the plain segmented Sieve of Eratosthenes in
  ``oracle.c`` (Fig. 1 of the paper, segmented as in Sec. 2.2, each prime
  starting at its square as in Sec. 1.1 and Sec. 2.4), one byte per integer,
  no wheel.  Loaded through ctypes from ``liboracle.so`` (built by ``build``).
* ``count_wide`` / ``primes_wide``: the same definition for values past 2^64
  (unsigned 128-bit arithmetic in ``oracle.c``; base primes listed by the
  64-bit sieve), for windows of the paper's next step beyond 64 bits (Sec. 6).
* ``brute``: trial division and deterministic Miller-Rabin, for pins.
* ``wheel``: the 6k+1/6k+5 index mapping (Sec. 2.1, Fig. 2) and the start
  index of Table 1 (Sec. 3), both as the paper states them and as their plain
  definition, plus the closed-form number of marks a prime makes on a range.

Ranges are half-open, [lo, hi), everywhere.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

from . import brute, wheel  # noqa: F401  (re-exported submodules)

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile ``liboracle.so`` with gcc (host code only, no HIP)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(
            ["gcc", "-O2", "-std=c11", "-Wall", "-Wextra", "-shared", "-fPIC", "-pthread",
             _SRC, "-o", tmp])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        lib = ctypes.CDLL(_LIB)
        lib.oracle_isqrt.restype = ctypes.c_uint64
        lib.oracle_isqrt.argtypes = [ctypes.c_uint64]
        lib.oracle_count.restype = ctypes.c_int64
        lib.oracle_count.argtypes = [ctypes.c_uint64, ctypes.c_uint64, ctypes.c_int]
        lib.oracle_list.restype = ctypes.c_int64
        lib.oracle_list.argtypes = [ctypes.c_uint64, ctypes.c_uint64, ctypes.c_void_p,
                                    ctypes.c_uint64, ctypes.c_int, ctypes.c_int]
        lib.oracle_simple_primes.restype = ctypes.c_int64
        lib.oracle_simple_primes.argtypes = [ctypes.c_uint64, ctypes.c_void_p, ctypes.c_uint64]
        lib.oracle_wide.restype = ctypes.c_int64
        lib.oracle_wide.argtypes = [ctypes.c_uint64] * 4 + [ctypes.c_void_p, ctypes.c_uint64, ctypes.c_int]
        _lib = lib
    return _lib


def default_threads() -> int:
    """Host threads the oracle uses by default (all visible cores)."""
    try:
        return max(1, len(os.sched_getaffinity(0)))
    except AttributeError:  # pragma: no cover
        return max(1, os.cpu_count() or 1)


def isqrt(n: int) -> int:
    """floor(sqrt(n)) by integer Newton iteration (oracle.c)."""
    return int(_load().oracle_isqrt(n))


def count(lo: int, hi: int, threads: int | None = None) -> int:
    """Number of primes in [lo, hi)."""
    if threads is None:
        threads = default_threads()
    r = _load().oracle_count(lo, hi, threads)
    if r < 0:
        raise ValueError("oracle_count(%d, %d) failed with %d" % (lo, hi, r))
    return int(r)


def primes(lo: int, hi: int, elem_bytes: int = 8, threads: int | None = None) -> np.ndarray:
    """Primes of [lo, hi) in increasing order, as uint32 (elem_bytes=4) or uint64."""
    if threads is None:
        threads = default_threads()
    lib = _load()
    n = lib.oracle_count(lo, hi, threads)
    if n < 0:
        raise ValueError("oracle_count(%d, %d) failed with %d" % (lo, hi, n))
    out = np.empty(max(n, 1), dtype=np.uint32 if elem_bytes == 4 else np.uint64)
    r = lib.oracle_list(lo, hi, out.ctypes.data, n, elem_bytes, threads)
    if r != n:
        raise ValueError("oracle_list(%d, %d) returned %d, expected %d" % (lo, hi, r, n))
    return out[:n]


def simple_primes(limit: int) -> np.ndarray:
    """Primes <= limit from the unsegmented sieve of Fig. 1 (uint32)."""
    lib = _load()
    n = lib.oracle_simple_primes(limit, None, 0)
    if n < 0:
        raise ValueError("oracle_simple_primes(%d) failed" % limit)
    out = np.empty(max(n, 1), dtype=np.uint32)
    lib.oracle_simple_primes(limit, out.ctypes.data, n)
    return out[:n]


def _halves(x: int):
    return x & (2 ** 64 - 1), x >> 64


def count_wide(lo: int, hi: int, threads: int | None = None) -> int:
    """Number of primes in [lo, hi) for values up to 2^128 (hi - lo < 2^63,
    isqrt(hi - 1) < 2^40)."""
    if threads is None:
        threads = default_threads()
    r = _load().oracle_wide(*_halves(lo), *_halves(hi), None, 0, threads)
    if r < 0:
        raise ValueError("oracle_wide(%d, %d) failed with %d" % (lo, hi, r))
    return int(r)


def primes_wide(lo: int, hi: int, threads: int | None = None) -> np.ndarray:
    """Primes of [lo, hi) beyond 64 bits, as an (n, 2) uint64 array of
    (low half, high half) per prime, in increasing order."""
    if threads is None:
        threads = default_threads()
    n = count_wide(lo, hi, threads)
    out = np.empty((max(n, 1), 2), dtype=np.uint64)
    r = _load().oracle_wide(*_halves(lo), *_halves(hi), out.ctypes.data, n, threads)
    if r != n:
        raise ValueError("oracle_wide list of [%d, %d) returned %d, expected %d" % (lo, hi, r, n))
    return out[:n]
