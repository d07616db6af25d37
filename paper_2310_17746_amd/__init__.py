"""MI355X segmented wheel sieve: Python binding of libsieve.so.

Argument marshalling only: every step of the sieve runs in the library's HIP
kernels.  PyTorch supplies device memory for list outputs and the HIP stream
they are ordered on.  Importing this package does not load the library; the
first use does, and it raises if ``libsieve.so`` was not built (there is no
fallback path).

    from paper_2310_17746_amd import Sieve
    s = Sieve()                      # device 0, default parameters
    s.base_primes(10**6)             # resident primes <= 10^6
    s.count(2, 10**12 + 1)           # pi(10^12)
    t = s.list(10**9, 10**9 + 10**6) # torch tensor of uint64 primes on cuda
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

__all__ = ["Sieve", "Server", "Generator", "SieveError", "Params", "ListResult", "U128", "list_bound",
           "list_bound_wide", "wide_values", "wheel_start", "plan_range", "probe_lds",
           "lib_path", "load_library", "SIEVE_OK", "SIEVE_E_CAPACITY", "SIEVE_E_LIMIT",
           "STATIC_MAX_RANGES", "WIDE_MIN_LO", "WIDE_MAX_SPAN", "WIDE_MAX_BASE"]

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libsieve.so")
_lib = None

SIEVE_OK = 0
SIEVE_E_INVAL = -1
SIEVE_E_RANGE = -2
SIEVE_E_CAPACITY = -3
SIEVE_E_DTYPE = -4
SIEVE_E_NOMEM = -5
SIEVE_E_DEVICE = -6
SIEVE_E_BUSY = -7
SIEVE_E_CANCELLED = -8
SIEVE_E_IO = -9
SIEVE_E_LIMIT = -10
STATIC_MAX_RANGES = 1024        # ranges per sieve_count_batch_static call
WIDE_MIN_LO = 1 << 40            # windows of the wide calls start here or later
WIDE_MAX_SPAN = 1 << 40          # and span at most this many integers
WIDE_MAX_BASE = 1 << 36          # largest base-prime limit of the wide calls
PRESIEVE_NONE = 0xFFFFFFFF
BUCKET_NEVER = 0xFFFFFFFF
BUCKET_EXACT = 1
BUCKET_TINY = 2
SKIP_ALL = 1
SKIP_NONE = 2
SKIP_SPLIT = 3
DENSE_NEVER = 0xFFFFFFFF
VISIT_COSTLY_FIRST, VISIT_REVERSED, VISIT_SHUFFLED = 0, 1, 2

_u64 = ctypes.c_uint64
_p = ctypes.c_void_p


class Params(ctypes.Structure):
    """sieve_params (include/sieve.h); zero fields select the defaults."""
    _fields_ = [("segment_bytes", ctypes.c_uint32), ("block_threads", ctypes.c_uint32),
                ("presieve_groups", ctypes.c_uint32), ("split_hits", ctypes.c_uint32),
                ("bucket_threshold", ctypes.c_uint32), ("wg_per_cu", ctypes.c_uint32),
                ("use_graph", ctypes.c_uint32), ("bucket_slices", ctypes.c_uint32),
                ("cofactor_skip", ctypes.c_uint32), ("bucket_mem_mb", ctypes.c_uint32),
                ("dense_hits", ctypes.c_uint32), ("visit_order", ctypes.c_uint32),
                ("strip_tiles", ctypes.c_uint32), ("reserved", ctypes.c_uint32 * 3)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_ if k != "reserved"}


class U128(ctypes.Structure):
    """sieve_u128: a 128-bit value as two 64-bit halves."""
    _fields_ = [("lo", ctypes.c_uint64), ("hi", ctypes.c_uint64)]

    @classmethod
    def of(cls, v: int) -> "U128":
        if not 0 <= v < 1 << 128:
            raise ValueError("value outside [0, 2^128)")
        return cls(v & (2 ** 64 - 1), v >> 64)


class ServerParams(ctypes.Structure):
    """sieve_server_params (include/sieve.h); zero fields select the defaults."""
    _fields_ = [("out_budget_bytes", ctypes.c_uint64), ("max_active", ctypes.c_uint32),
                ("step_tiles", ctypes.c_uint32), ("quantum_tiles", ctypes.c_uint32),
                ("elem_bytes", ctypes.c_uint32), ("max_queue", ctypes.c_uint32),
                ("overlap", ctypes.c_uint32), ("restart_walks", ctypes.c_uint32)]


class Completion(ctypes.Structure):
    _fields_ = [("tag", ctypes.c_uint64), ("count", ctypes.c_uint64), ("lo", ctypes.c_uint64),
                ("hi", ctypes.c_uint64), ("t_arrival_ns", ctypes.c_uint64),
                ("t_admit_ns", ctypes.c_uint64), ("t_done_ns", ctypes.c_uint64),
                ("status", ctypes.c_int32), ("mode", ctypes.c_int32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class ServerStats(ctypes.Structure):
    _fields_ = [(k, ctypes.c_uint64) for k in ("steps", "tiles", "ints", "completed", "busy_ns",
                                               "elapsed_ns", "arena_peak_bytes", "queued", "active",
                                               "bucket_steps", "overlap_steps", "resumed_walks",
                                               "walk_bytes")]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class SieveError(RuntimeError):
    def __init__(self, code: int, what: str):
        self.code = code
        super().__init__("%s: %s (%d)" % (what, load_library().sieve_strerror(code).decode(), code))


def lib_path() -> str:
    return _LIB_PATH


def load_library():
    """Loads libsieve.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        raise ImportError("libsieve.so not built: run __graft_entry__.build() "
                          "(python -c 'import __graft_entry__ as g; g.build()')")
    lib = ctypes.CDLL(_LIB_PATH)
    sig = {
        "sieve_default_params": (ctypes.c_int, [ctypes.POINTER(Params)]),
        "sieve_create": (ctypes.c_int, [ctypes.POINTER(_p), ctypes.c_int, ctypes.POINTER(Params)]),
        "sieve_destroy": (ctypes.c_int, [_p]),
        "sieve_get_params": (ctypes.c_int, [_p, ctypes.POINTER(Params)]),
        "sieve_base_primes": (ctypes.c_int, [_p, _u64, ctypes.POINTER(_u64)]),
        "sieve_base_limit": (ctypes.c_int, [_p, ctypes.POINTER(_u64)]),
        "sieve_count": (ctypes.c_int, [_p, _u64, _u64, ctypes.POINTER(_u64)]),
        "sieve_list": (ctypes.c_int, [_p, _u64, _u64, _p, _u64, ctypes.c_int,
                                      ctypes.POINTER(_u64), _p]),
        "sieve_count_batch": (ctypes.c_int, [_p, _p, _p, _u64, _p, _p]),
        "sieve_count_batch_static": (ctypes.c_int, [_p, _p, _p, _u64, _p, _p]),
        "sieve_list_batch": (ctypes.c_int, [_p, _p, _p, _p, _u64, _p, _p, _p, ctypes.c_int,
                                            _p, _p, _p]),
        "sieve_list_bound": (_u64, [_u64, _u64]),
        "sieve_base_primes_wide": (ctypes.c_int, [_p, _u64, ctypes.POINTER(_u64)]),
        "sieve_ext_limit": (ctypes.c_int, [_p, ctypes.POINTER(_u64)]),
        "sieve_count_wide": (ctypes.c_int, [_p, ctypes.POINTER(U128), ctypes.POINTER(U128),
                                            ctypes.POINTER(_u64), _p]),
        "sieve_list_wide": (ctypes.c_int, [_p, ctypes.POINTER(U128), ctypes.POINTER(U128), _p, _u64,
                                           ctypes.POINTER(_u64), _p]),
        "sieve_wheel_start": (ctypes.c_int, [_u64, _u64, _u64, ctypes.POINTER(ctypes.c_int64),
                                             ctypes.POINTER(ctypes.c_int64)]),
        "sieve_plan_range": (ctypes.c_int, [_u64, _u64, ctypes.c_uint32, ctypes.POINTER(_u64),
                                            ctypes.POINTER(_u64), ctypes.POINTER(ctypes.c_uint32)]),
        "sieve_set_timing": (ctypes.c_int, [_p, ctypes.c_int]),
        "sieve_get_timing": (ctypes.c_int, [_p, ctypes.POINTER(ctypes.c_double),
                                            ctypes.POINTER(ctypes.c_double),
                                            ctypes.POINTER(ctypes.c_double), ctypes.POINTER(_u64)]),
        "sieve_probe_lds": (ctypes.c_int, [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                           ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double)]),
        "sieve_strerror": (ctypes.c_char_p, [ctypes.c_int]),
        "sieve_last_error": (ctypes.c_int, [_p]),
        "sieve_server_create": (ctypes.c_int, [_p, ctypes.POINTER(ServerParams), ctypes.POINTER(_p)]),
        "sieve_submit": (ctypes.c_int, [_p, _u64, _u64, ctypes.c_int, _u64]),
        "sieve_submit_at": (ctypes.c_int, [_p, _u64, _u64, ctypes.c_int, _u64, _u64]),
        "sieve_submit_out": (ctypes.c_int, [_p, _u64, _u64, ctypes.c_int, _p, _u64, _u64]),
        "sieve_poll": (ctypes.c_int, [_p, ctypes.POINTER(Completion), ctypes.c_int, ctypes.c_int,
                                      ctypes.POINTER(ctypes.c_int)]),
        "sieve_cancel": (ctypes.c_int, [_p, _u64]),
        "sieve_server_fetch": (ctypes.c_int, [_p, _u64, _p, _u64, ctypes.POINTER(_u64)]),
        "sieve_server_release": (ctypes.c_int, [_p, _u64]),
        "sieve_server_get_stats": (ctypes.c_int, [_p, ctypes.POINTER(ServerStats)]),
        "sieve_server_now_ns": (_u64, [_p]),
        "sieve_server_destroy": (ctypes.c_int, [_p]),
        "sieve_gen_create": (ctypes.c_int, [_p, _u64, ctypes.c_int, ctypes.POINTER(_p)]),
        "sieve_gen_next": (ctypes.c_int, [_p, _u64, _p, ctypes.POINTER(_u64), _p]),
        "sieve_gen_position": (ctypes.c_int, [_p, ctypes.POINTER(_u64)]),
        "sieve_gen_destroy": (ctypes.c_int, [_p]),
        "sieve_list_host": (ctypes.c_int, [_p, _u64, _u64, _p, _u64, ctypes.c_int, _u64,
                                           ctypes.POINTER(_u64)]),
        "sieve_write_files": (ctypes.c_int, [_p, _u64, _u64, ctypes.c_char_p, _u64, ctypes.c_int, _u64,
                                             ctypes.POINTER(_u64), ctypes.POINTER(_u64)]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


def _check(code: int, what: str) -> None:
    if code != SIEVE_OK:
        raise SieveError(code, what)


def list_bound(lo: int, hi: int) -> int:
    """Rigorous upper bound on the number of primes in [lo, hi)."""
    return int(load_library().sieve_list_bound(lo, hi))


def list_bound_wide(lo: int, hi: int) -> int:
    """The bound of list_bound for a wide window: it depends only on lo mod 6
    and hi - lo, so it is taken on a window of the same shape below 2^63."""
    if hi <= lo:
        return 0
    base = 6 << 37
    return list_bound(base + lo % 6, base + lo % 6 + (hi - lo))


def wide_values(t) -> list:
    """Python ints from a wide list (a tensor or array of shape (n, 2) whose
    rows hold the low and high 64-bit halves)."""
    a = t.cpu().numpy() if hasattr(t, "cpu") else np.asarray(t)
    a = a.view(np.uint64).reshape(-1, 2)
    return [int(h) << 64 | int(lo) for lo, h in a]


def wheel_start(p: int, base: int, M: int) -> tuple[int, int]:
    """Table 1 start indices (id_1, id_5) from the library's host-compiled code."""
    a, b = ctypes.c_int64(), ctypes.c_int64()
    _check(load_library().sieve_wheel_start(p, base, M, ctypes.byref(a), ctypes.byref(b)),
           "sieve_wheel_start")
    return a.value, b.value


def plan_range(lo: int, hi: int, segment_bytes: int) -> tuple[int, int, int]:
    """(ntiles, base, last_words) of the tile plan of [lo, hi)."""
    n, b, w = _u64(), _u64(), ctypes.c_uint32()
    _check(load_library().sieve_plan_range(lo, hi, segment_bytes, ctypes.byref(n), ctypes.byref(b),
                                           ctypes.byref(w)), "sieve_plan_range")
    return n.value, b.value, w.value


PROBE_MODES = {"or_linear": 0, "or_random": 1, "or_even": 2, "or_same": 3, "write_linear": 4,
               "write_random": 5, "write8_random": 6, "read_random": 7}


def probe_lds(mode: str, iters: int = 4096, wg_per_cu: int = 1, device: int = 0) -> tuple[float, float]:
    """LDS probe (include/sieve_probe.h): (lane operations per second, kernel ms)."""
    ops, ms = ctypes.c_double(), ctypes.c_double()
    code = load_library().sieve_probe_lds(device, PROBE_MODES[mode], iters, wg_per_cu,
                                          ctypes.byref(ops), ctypes.byref(ms))
    if code != 0:
        raise SieveError(code, "sieve_probe_lds")
    return ops.value, ms.value


def _torch():
    import torch
    return torch


def _dtype_for(elem_bytes: int):
    torch = _torch()
    return torch.int32 if elem_bytes == 4 else torch.int64


def _stream_handle(stream):
    if stream is None:
        return None
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


def _sync(stream) -> None:
    """Waits for a torch stream (or a raw hipStream_t handle)."""
    torch = _torch()
    if isinstance(stream, int):
        stream = torch.cuda.ExternalStream(stream)
    stream.synchronize()


class ListResult:
    """A stream-ordered list call: `out` is filled and `count` is valid once
    the stream has reached the end of the job (after it synchronizes).  Keep
    this object alive until then: the library writes the count into it."""

    def __init__(self, out, stream):
        self.out = out
        self.stream = stream
        self._n = _u64()

    @property
    def count(self) -> int:
        return self._n.value

    def primes(self):
        """The filled prefix of `out` (after the stream has synchronized)."""
        return self.out[: min(self._n.value, self.out.numel())]


class Sieve:
    """A sieve context on one GPU (resident base primes, scratch, stream)."""

    def __init__(self, device: int = 0, params: Params | dict | None = None):
        lib = load_library()
        self._lib = lib
        self.device = device
        p = None
        if params is not None:
            if isinstance(params, dict):
                q = Params()
                for k, v in params.items():
                    setattr(q, k, v)
                params = q
            p = ctypes.byref(params)
        h = _p()
        _check(lib.sieve_create(ctypes.byref(h), device, p), "sieve_create")
        self._h = h

    # -- lifetime ----------------------------------------------------------
    def close(self) -> None:
        if getattr(self, "_h", None):
            self._lib.sieve_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    # -- queries -----------------------------------------------------------
    @property
    def params(self) -> Params:
        q = Params()
        _check(self._lib.sieve_get_params(self._h, ctypes.byref(q)), "sieve_get_params")
        return q

    @property
    def base_limit(self) -> int:
        v = _u64()
        _check(self._lib.sieve_base_limit(self._h, ctypes.byref(v)), "sieve_base_limit")
        return v.value

    def base_primes(self, limit: int) -> int:
        """Makes all primes <= limit resident; returns how many (>= 5) are."""
        n = _u64()
        _check(self._lib.sieve_base_primes(self._h, limit, ctypes.byref(n)), "sieve_base_primes")
        return n.value

    def ensure_base_for(self, hi: int) -> None:
        """Makes the base primes cover isqrt(hi - 1)."""
        import math
        need = math.isqrt(max(hi - 1, 0))
        if need > self.base_limit:
            self.base_primes(need)

    @property
    def ext_limit(self) -> int:
        v = _u64()
        _check(self._lib.sieve_ext_limit(self._h, ctypes.byref(v)), "sieve_ext_limit")
        return v.value

    def base_primes_wide(self, limit: int) -> int:
        """Makes all primes <= limit (<= 2^36) available to the wide calls:
        resident below 2^32, an extension list above; returns how many."""
        n = _u64()
        _check(self._lib.sieve_base_primes_wide(self._h, limit, ctypes.byref(n)), "sieve_base_primes_wide")
        return n.value

    def ensure_base_wide_for(self, hi: int) -> None:
        """Makes the wide calls' base primes cover isqrt(hi - 1)."""
        import math
        need = math.isqrt(max(hi - 1, 0))
        if need > 1 << 32:  # 2^32 itself is not prime
            if need > self.ext_limit:
                self.base_primes_wide(need)
        elif min(need, (1 << 32) - 1) > self.base_limit:
            self.base_primes(min(need, (1 << 32) - 1))

    def count_wide(self, lo: int, hi: int, stream=None) -> int:
        """Number of primes in [lo, hi), 2^40 <= lo, hi - lo <= 2^40, values up
        to 2^128 (the base primes must cover isqrt(hi - 1))."""
        c = _u64()
        a, b = U128.of(lo), U128.of(hi)
        _check(self._lib.sieve_count_wide(self._h, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c),
                                          _stream_handle(stream)), "sieve_count_wide")
        return c.value

    def list_wide(self, lo: int, hi: int, out=None, stream=None):
        """Primes of the window [lo, hi) as an int64 tensor of shape (n, 2) on
        the context's GPU: row k holds the low and high 64-bit halves of the
        k-th prime (bit for bit).  With `out` (shape (cap, 2), int64) given,
        a view of its filled prefix is returned."""
        torch = _torch()
        if out is None:
            out = torch.empty((max(list_bound_wide(lo, hi), 1), 2), dtype=torch.int64,
                              device="cuda:%d" % self.device)
        if out.dtype != torch.int64 or out.dim() != 2 or out.shape[1] != 2 or not out.is_contiguous():
            raise ValueError("out must be a contiguous int64 tensor of shape (cap, 2)")
        n = _u64()
        a, b = U128.of(lo), U128.of(hi)
        code = self._lib.sieve_list_wide(self._h, ctypes.byref(a), ctypes.byref(b), out.data_ptr(),
                                         out.shape[0], ctypes.byref(n), _stream_handle(stream))
        if code == SIEVE_E_CAPACITY:
            raise SieveError(code, "sieve_list_wide needs %d elements" % n.value)
        _check(code, "sieve_list_wide")
        return out[: n.value]

    def count(self, lo: int, hi: int) -> int:
        c = _u64()
        _check(self._lib.sieve_count(self._h, lo, hi, ctypes.byref(c)), "sieve_count")
        return c.value

    def list(self, lo: int, hi: int, out=None, elem_bytes: int | None = None, stream=None):
        """Primes of [lo, hi) as a torch tensor on the context's GPU.

        The tensor has dtype int32 (elem_bytes=4) or int64 holding the
        unsigned values bit for bit.  With `out` given, the primes are
        written into it and a view of the filled prefix is returned.
        """
        torch = _torch()
        if elem_bytes is None:
            elem_bytes = 4 if hi <= 2 ** 32 else 8
        if out is None:
            out = torch.empty(max(list_bound(lo, hi), 1), dtype=_dtype_for(elem_bytes),
                              device="cuda:%d" % self.device)
        if out.element_size() != elem_bytes or not out.is_contiguous():
            raise ValueError("out must be contiguous with %d-byte elements" % elem_bytes)
        n = _u64()
        code = self._lib.sieve_list(self._h, lo, hi, out.data_ptr(), out.numel(), elem_bytes,
                                    ctypes.byref(n), _stream_handle(stream))
        if code == SIEVE_E_CAPACITY:
            raise SieveError(code, "sieve_list needs %d elements" % n.value)
        _check(code, "sieve_list")
        if stream is not None:
            _sync(stream)  # the call was stream-ordered: n is written when the stream gets there
            if n.value > out.numel():
                raise SieveError(SIEVE_E_CAPACITY, "sieve_list needs %d elements" % n.value)
        return out[: n.value]

    def list_async(self, lo: int, hi: int, out, elem_bytes: int, stream) -> "ListResult":
        """Enqueues the list of [lo, hi) into `out` on `stream` and returns at
        once (a job that needs the bucket sieve waits for the stream first).
        The returned ListResult's count and primes() are valid after the
        stream synchronizes; a count above out.numel() means nothing was
        written."""
        if out.element_size() != elem_bytes or not out.is_contiguous():
            raise ValueError("out must be contiguous with %d-byte elements" % elem_bytes)
        r = ListResult(out, stream)
        _check(self._lib.sieve_list(self._h, lo, hi, out.data_ptr(), out.numel(), elem_bytes,
                                    ctypes.byref(r._n), _stream_handle(stream)), "sieve_list")
        return r

    def list_host(self, lo: int, hi: int, elem_bytes: int = 8, out=None, piece_elems: int = 0):
        """Primes of [lo, hi) streamed into host memory.

        `out` may be a numpy array or a (pinned) CPU torch tensor with
        elem_bytes-byte elements; by default a numpy array of the rigorous
        bound is allocated.  Returns the filled prefix.
        """
        if out is None:
            out = np.empty(max(list_bound(lo, hi), 1), dtype=np.uint32 if elem_bytes == 4 else np.uint64)
        if isinstance(out, np.ndarray):
            if out.itemsize != elem_bytes or not out.flags["C_CONTIGUOUS"]:
                raise ValueError("out must be contiguous with %d-byte elements" % elem_bytes)
            ptr, cap = out.ctypes.data, out.size
        else:
            if out.element_size() != elem_bytes or not out.is_contiguous() or out.is_cuda:
                raise ValueError("out must be a contiguous host tensor with %d-byte elements" % elem_bytes)
            ptr, cap = out.data_ptr(), out.numel()
        n = _u64()
        code = self._lib.sieve_list_host(self._h, lo, hi, ptr, cap, elem_bytes, piece_elems, ctypes.byref(n))
        if code == SIEVE_E_CAPACITY:
            raise SieveError(code, "sieve_list_host needs %d elements" % n.value)
        _check(code, "sieve_list_host")
        return out[: n.value]

    def write_files(self, lo: int, hi: int, path_prefix: str, primes_per_file: int = 0,
                    elem_bytes: int = 8, piece_elems: int = 0) -> tuple[int, int]:
        """Writes the primes of [lo, hi) to <prefix>.000000, ...; returns (count, files)."""
        n, nf = _u64(), _u64()
        _check(self._lib.sieve_write_files(self._h, lo, hi, os.fsencode(path_prefix), primes_per_file,
                                           elem_bytes, piece_elems, ctypes.byref(n), ctypes.byref(nf)),
               "sieve_write_files")
        return n.value, nf.value

    def generator(self, start: int = 0, elem_bytes: int = 8) -> "Generator":
        """An incremental generator of the primes >= start (see Generator)."""
        return Generator(self, start, elem_bytes)

    def count_list(self, lo: int, hi: int, elem_bytes: int = 8) -> int:
        """Count through the list path without an output buffer (cap 0)."""
        n = _u64()
        code = self._lib.sieve_list(self._h, lo, hi, None, 0, elem_bytes, ctypes.byref(n), None)
        if code not in (SIEVE_OK, SIEVE_E_CAPACITY):
            _check(code, "sieve_list")
        return n.value

    def count_batch(self, lo, hi, stream=None, sync: bool = True) -> np.ndarray:
        """Counts of many ranges in one job.  With a stream and sync=False the
        call is stream-ordered: the returned array is filled when the stream
        reaches the end of the job (keep it until the stream synchronizes)."""
        lo = np.ascontiguousarray(lo, dtype=np.uint64)
        hi = np.ascontiguousarray(hi, dtype=np.uint64)
        if lo.shape != hi.shape:
            raise ValueError("lo and hi differ in shape")
        counts = np.zeros(lo.shape, dtype=np.uint64)
        _check(self._lib.sieve_count_batch(self._h, lo.ctypes.data, hi.ctypes.data, lo.size,
                                           counts.ctypes.data, _stream_handle(stream)),
               "sieve_count_batch")
        if stream is not None and sync:
            _sync(stream)
        return counts

    def count_batch_static(self, lo, hi, stream=None) -> np.ndarray:
        """As count_batch, through the entry point that allocates nothing
        (fixed device scratch; at most STATIC_MAX_RANGES ranges per call)."""
        lo = np.ascontiguousarray(lo, dtype=np.uint64)
        hi = np.ascontiguousarray(hi, dtype=np.uint64)
        if lo.shape != hi.shape:
            raise ValueError("lo and hi differ in shape")
        counts = np.zeros(lo.shape, dtype=np.uint64)
        _check(self._lib.sieve_count_batch_static(self._h, lo.ctypes.data, hi.ctypes.data, lo.size,
                                                  counts.ctypes.data, _stream_handle(stream)),
               "sieve_count_batch_static")
        return counts

    def list_batch(self, lo, hi, mode, out, off, cap, elem_bytes: int = 8, stream=None, sync: bool = True):
        """Mixed batch; returns (counts, status) as numpy arrays (with a stream
        and sync=False: filled when the stream reaches the end of the job)."""
        lo = np.ascontiguousarray(lo, dtype=np.uint64)
        hi = np.ascontiguousarray(hi, dtype=np.uint64)
        mode = np.ascontiguousarray(mode, dtype=np.uint8)
        off = np.ascontiguousarray(off, dtype=np.uint64)
        cap = np.ascontiguousarray(cap, dtype=np.uint64)
        n = lo.size
        counts = np.zeros(n, dtype=np.uint64)
        status = np.zeros(n, dtype=np.int32)
        optr = out.data_ptr() if out is not None else None
        _check(self._lib.sieve_list_batch(self._h, lo.ctypes.data, hi.ctypes.data, mode.ctypes.data,
                                          n, optr, off.ctypes.data, cap.ctypes.data, elem_bytes,
                                          counts.ctypes.data, status.ctypes.data,
                                          _stream_handle(stream)), "sieve_list_batch")
        if stream is not None and sync:
            _sync(stream)
        return counts, status

    # -- measurement -------------------------------------------------------
    def set_timing(self, on: bool = True) -> None:
        _check(self._lib.sieve_set_timing(self._h, 1 if on else 0), "sieve_set_timing")

    def timing(self) -> tuple[float, float, int]:
        """(sieve kernel ms, finalize+compaction ms, jobs) summed since set_timing."""
        a, b, c, n = self.timing_all()
        return a, b, n

    def timing_all(self) -> tuple[float, float, float, int]:
        """(sieve ms, finalize+compaction ms, bucket-sieve ms, jobs) since set_timing."""
        a, b, c, n = ctypes.c_double(), ctypes.c_double(), ctypes.c_double(), _u64()
        _check(self._lib.sieve_get_timing(self._h, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c),
                                          ctypes.byref(n)), "sieve_get_timing")
        return a.value, b.value, c.value, n.value


class Generator:
    """Hands out the primes from `start` on, n at a time, as device tensors.

    Keeps a reference to its Sieve; the two must not be used concurrently.
    """

    def __init__(self, sieve: "Sieve", start: int = 0, elem_bytes: int = 8):
        self._sieve = sieve
        self._lib = sieve._lib
        self.elem_bytes = elem_bytes
        h = _p()
        _check(self._lib.sieve_gen_create(sieve._h, start, elem_bytes, ctypes.byref(h)), "sieve_gen_create")
        self._h = h

    def close(self) -> None:
        if getattr(self, "_h", None):
            self._lib.sieve_gen_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    @property
    def position(self) -> int:
        v = _u64()
        _check(self._lib.sieve_gen_position(self._h, ctypes.byref(v)), "sieve_gen_position")
        return v.value

    def next(self, n: int, out=None, stream=None):
        """The next n primes (fewer at the end of the value domain)."""
        torch = _torch()
        if out is None:
            out = torch.empty(max(n, 1), dtype=_dtype_for(self.elem_bytes),
                              device="cuda:%d" % self._sieve.device)
        if out.element_size() != self.elem_bytes or not out.is_contiguous() or out.numel() < n:
            raise ValueError("out must be contiguous with room for %d %d-byte elements" % (n, self.elem_bytes))
        got = _u64()
        _check(self._lib.sieve_gen_next(self._h, n, out.data_ptr(), ctypes.byref(got), _stream_handle(stream)),
               "sieve_gen_next")
        return out[: got.value]


class Server:
    """Continuous-batching range-query server on a Sieve context.

    While the server exists the context must not be used for other calls.
    """

    def __init__(self, sieve: "Sieve", **params):
        self._sieve = sieve
        self._lib = sieve._lib
        p = ServerParams()
        for k, v in params.items():
            setattr(p, k, v)
        h = _p()
        _check(self._lib.sieve_server_create(sieve._h, ctypes.byref(p), ctypes.byref(h)),
               "sieve_server_create")
        self._h = h
        self.elem_bytes = params.get("elem_bytes", 8) or 8

    def close(self) -> None:
        if getattr(self, "_h", None):
            self._lib.sieve_server_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def now_ns(self) -> int:
        return int(self._lib.sieve_server_now_ns(self._h))

    def submit(self, lo: int, hi: int, mode: int, tag: int, at_ns: int | None = None, out=None) -> None:
        """Queues [lo, hi) (mode 0 count, 1 list).  With `out` (a contiguous
        device tensor of the server's element size) a list goes straight
        into it, at most out.numel() elements, instead of the arena."""
        if out is not None:
            if at_ns is not None:
                raise ValueError("a scheduled arrival takes the arena output")
            if not out.is_contiguous():
                raise ValueError("out must be contiguous")
            code = self._lib.sieve_submit_out(self._h, lo, hi, mode, out.data_ptr(), out.numel(), tag)
        elif at_ns is None:
            code = self._lib.sieve_submit(self._h, lo, hi, mode, tag)
        else:
            code = self._lib.sieve_submit_at(self._h, lo, hi, mode, tag, at_ns)
        _check(code, "sieve_submit")

    def poll(self, max_items: int = 4096, wait_ms: int = 0) -> list[dict]:
        buf = (Completion * max_items)()
        n = ctypes.c_int()
        _check(self._lib.sieve_poll(self._h, buf, max_items, wait_ms, ctypes.byref(n)), "sieve_poll")
        return [buf[i].as_dict() for i in range(n.value)]

    def cancel(self, tag: int) -> int:
        return int(self._lib.sieve_cancel(self._h, tag))

    def fetch(self, tag: int, count: int, device: bool = True):
        """Copies a finished list result into a new tensor and frees its space."""
        torch = _torch()
        dev = "cuda:%d" % self._sieve.device if device else "cpu"
        out = torch.empty(max(count, 1), dtype=_dtype_for(self.elem_bytes), device=dev)
        n = _u64()
        _check(self._lib.sieve_server_fetch(self._h, tag, out.data_ptr(), out.numel(), ctypes.byref(n)),
               "sieve_server_fetch")
        return out[: n.value]

    def release(self, tag: int) -> None:
        _check(self._lib.sieve_server_release(self._h, tag), "sieve_server_release")

    def stats(self) -> dict:
        st = ServerStats()
        _check(self._lib.sieve_server_get_stats(self._h, ctypes.byref(st)), "sieve_server_get_stats")
        return st.as_dict()
