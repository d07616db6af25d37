"""GPU parity of the incremental generator and the streaming outputs.

The generator (incremental generation, Sec. 2.4) and the host / file streams
(the Prime Number Data Store of Sec. 4 written out as Sec. 6 proposes) go
through the C ABI and are compared bit-exactly with the oracle's lists of the
same ranges.
"""
import ctypes
import os

import numpy as np
import pytest

import oracle

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
pkg = pytest.importorskip("paper_2310_17746_amd")


def _u(t, elem_bytes):
    a = t.cpu().numpy()
    return a.view(np.uint32 if elem_bytes == 4 else np.uint64)


@pytest.fixture(scope="module")
def sv():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    s = pkg.Sieve(0)
    s.base_primes(1 << 20)
    yield s
    s.close()


def test_generator_from_zero_in_uneven_steps(sv):
    steps = [1, 2, 10, 1000, 0, 12345, 1 << 20, 777, 3]
    want = oracle.primes(0, 20_000_000)
    with sv.generator(0, 8) as g:
        assert g.position == 0
        got = []
        for n in steps:
            t = g.next(n)
            assert t.numel() == n
            got.append(_u(t, 8))
            total = sum(len(x) for x in got)
            if total:
                assert g.position == int(want[total - 1]) + 1
    got = np.concatenate(got)
    assert np.array_equal(got, want[: len(got)])


@pytest.mark.parametrize("start", [0, 1, 2, 3, 4, 5, 6, 7, 24, 25, 10 ** 9 + 7])
def test_generator_start_values(sv, start):
    with sv.generator(start, 8) as g:
        got = _u(g.next(5), 8)
    want = oracle.primes(start, start + 1000)[:5]
    assert np.array_equal(got, want), (start, got, want)


def test_generator_grows_base_primes_from_1e12(sv):
    start = 10 ** 12 - 1000
    with pkg.Sieve(0) as s:
        assert s.base_limit == 0
        with s.generator(start, 8) as g:
            a = _u(g.next(1 << 21), 8)
            b = _u(g.next((1 << 21) + 11), 8)
            pos = g.position
        assert s.base_limit >= 10 ** 6
    got = np.concatenate([a, b])
    assert pos == int(got[-1]) + 1
    want = oracle.primes(start, pos)
    assert np.array_equal(got, want)


def test_generator_u32_reaches_domain_end(sv):
    start = (1 << 32) - 10 ** 6
    want = oracle.primes(start, 1 << 32)
    with sv.generator(start, 4) as g:
        t = g.next(10 ** 6)
        assert t.numel() == len(want)
        assert np.array_equal(_u(t, 4).astype(np.uint64), want)
        assert g.position == 1 << 32
        assert g.next(10).numel() == 0
    with pytest.raises(pkg.SieveError):
        sv.generator((1 << 32) + 1, 4)


@pytest.mark.parametrize("elem_bytes", [4, 8])
def test_list_host_pageable_many_pieces(sv, elem_bytes):
    lo, hi = 10 ** 9 - 12345, 10 ** 9 + 3 * 10 ** 7
    got = sv.list_host(lo, hi, elem_bytes=elem_bytes, piece_elems=100_000)
    want = oracle.primes(lo, hi)
    assert np.array_equal(got.astype(np.uint64), want)


def test_list_host_pinned_direct(sv):
    lo, hi = 10 ** 12, 10 ** 12 + 2 * 10 ** 8
    out = torch.empty(pkg.list_bound(lo, hi), dtype=torch.int64, pin_memory=True)
    got = sv.list_host(lo, hi, elem_bytes=8, out=out, piece_elems=1 << 20)
    want = oracle.primes(lo, hi)
    assert np.array_equal(got.numpy().view(np.uint64), want)


def test_list_host_default_pieces_and_capacity(sv):
    lo, hi = 0, 10 ** 9 + 1
    want_n = 50_847_534
    got = sv.list_host(lo, hi, elem_bytes=4)
    assert len(got) == want_n
    assert np.array_equal(got[:1000].astype(np.uint64), oracle.primes(0, 7920))
    assert np.array_equal(got[-1000:].astype(np.uint64), oracle.primes(10 ** 9 - 30000, hi)[-1000:])
    lib = pkg.load_library()
    small = np.zeros(1000, dtype=np.uint64)
    n = ctypes.c_uint64()
    code = lib.sieve_list_host(sv._h, 10 ** 6, 2 * 10 ** 6, small.ctypes.data, small.size, 8, 256,
                               ctypes.byref(n))
    assert code == pkg.SIEVE_E_CAPACITY
    assert n.value == oracle.count(10 ** 6, 2 * 10 ** 6)
    code = lib.sieve_list_host(sv._h, 0, 100, small.ctypes.data, small.size, 8, 255, ctypes.byref(n))
    assert code == pkg.SIEVE_E_INVAL
    code = lib.sieve_list_host(sv._h, 0, (1 << 32) + 1, small.ctypes.data, small.size, 4, 0, ctypes.byref(n))
    assert code == pkg.SIEVE_E_DTYPE


def test_write_files(sv, tmp_path):
    lo, hi = 0, 10 ** 7 + 1
    prefix = str(tmp_path / "primes")
    n, nf = sv.write_files(lo, hi, prefix, primes_per_file=100_000, elem_bytes=4, piece_elems=50_000)
    want = oracle.primes(lo, hi)
    assert n == len(want) == 664_579
    assert nf == 7
    parts = []
    for i in range(nf):
        path = "%s.%06d" % (prefix, i)
        size = os.path.getsize(path)
        assert size == (100_000 if i < nf - 1 else n - 100_000 * (nf - 1)) * 4
        parts.append(np.fromfile(path, dtype="<u4"))
    assert not os.path.exists("%s.%06d" % (prefix, nf))
    assert np.array_equal(np.concatenate(parts).astype(np.uint64), want)
    # An empty range creates no file; an unwritable prefix reports SIEVE_E_IO.
    assert sv.write_files(10, 10, str(tmp_path / "empty")) == (0, 0)
    assert not os.path.exists(str(tmp_path / "empty.000000"))
    with pytest.raises(pkg.SieveError) as e:
        sv.write_files(0, 1000, str(tmp_path / "no_such_dir" / "p"))
    assert e.value.code == pkg.SIEVE_E_IO
