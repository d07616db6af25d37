"""The allocation-free batched count (sieve_count_batch_static, fixed device
scratch) against the ordinary batched count (sieve_count_batch) through the
C ABI: bit-exact counts on two calls in a row, the second with fewer and
different ranges, so that the scratch holds the first call's contents when
the second starts.  Requests beyond the fixed scratch are refused before any
device work, and the base primes are never grown by this entry point."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
pkg = pytest.importorskip("paper_2310_17746_amd")
from paper_2310_17746_amd import workloads  # noqa: E402


def test_static_batch_equals_batch_on_two_calls():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    lo, hi, _ = workloads.batch_ranges(0)
    n1 = pkg.STATIC_MAX_RANGES
    a_lo, a_hi = lo[:n1].copy(), hi[:n1].copy()
    # degenerate ranges in the first call: empty, the primes 2 and 3, the value 1
    a_lo[:4] = [0, 0, 7, 1]
    a_hi[:4] = [0, 4, 7, 2]
    b_lo, b_hi = lo[n1:n1 + 300], hi[n1:n1 + 300]
    print("static batch: %d then %d ranges from the seed-0 batch" % (n1, len(b_lo)), flush=True)
    with pkg.Sieve(0) as s:
        s.ensure_base_for(int(max(a_hi.max(), b_hi.max())))
        want_a = s.count_batch(a_lo, a_hi)
        want_b = s.count_batch(b_lo, b_hi)
        got_a = s.count_batch_static(a_lo, a_hi)
        got_b = s.count_batch_static(b_lo, b_hi, stream=torch.cuda.current_stream())
        assert list(want_a[:4]) == [0, 2, 0, 0]
        bad = np.nonzero(got_a != want_a)[0]
        assert len(bad) == 0, [(int(a_lo[i]), int(a_hi[i]), int(got_a[i]), int(want_a[i])) for i in bad[:5]]
        bad = np.nonzero(got_b != want_b)[0]
        assert len(bad) == 0, [(int(b_lo[i]), int(b_hi[i]), int(got_b[i]), int(want_b[i])) for i in bad[:5]]


def test_static_batch_limits():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    with pkg.Sieve(0) as s:
        s.base_primes(1000)
        n = pkg.STATIC_MAX_RANGES + 1
        with pytest.raises(pkg.SieveError) as e:
            s.count_batch_static(np.zeros(n, dtype=np.uint64), np.full(n, 100, dtype=np.uint64))
        assert e.value.code == pkg.SIEVE_E_LIMIT
        # base primes cover isqrt(hi - 1) <= 1000 only; the call does not grow them
        with pytest.raises(pkg.SieveError) as e:
            s.count_batch_static([10 ** 7], [10 ** 7 + 10 ** 6])
        assert e.value.code == -2  # SIEVE_E_RANGE
        assert s.base_limit == 1000
        assert len(s.count_batch_static([], [])) == 0
        assert list(s.count_batch_static([0, 100], [100, 1000])) == [25, 143]
