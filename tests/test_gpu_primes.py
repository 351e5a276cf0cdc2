"""GPU tests of the prime subsequence (Section 3.2): the prime sieve and the
walks over primes only, against the oracle's trial division and full-period
walk.  Counts are integers: every comparison is exact."""
import sys

import numpy as np
import pytest

import oracle
import paper_2507_06579_amd as eis

pytestmark = pytest.mark.gpu


def _say(msg):
    print(f"[gpu-primes] {msg}", flush=True)
    sys.stdout.flush()


@pytest.mark.parametrize("a,b", [(0, 200000), (5, 6), (0, 14), (999000, 1001000),
                                 (10**6, 10**6 + 400000), (10**9, 10**9 + 200000),
                                 (10**11 - 100000, 10**11), (10**12 - 80000, 10**12)])
def test_prime_counts_against_oracle(a, b):
    with eis.Context() as c:
        _say(f"primes in [{a}, {b})")
        got = c.eis_count_set(eis.EIS_SET_PRIME, a, b)
    assert got == oracle.classify_primes(a, b), (a, b)


def test_prime_sieve_keeps_sieving_primes_themselves():
    # the primes p <= 10^3 with p = 5 (mod 8) sieve [0, 10^6) and must survive
    with eis.Context(method=eis.Method.BABY) as c:
        n_p, _ = c.eis_count_set(eis.EIS_SET_PRIME, 0, 10**6)
    assert n_p == sum(1 for p in range(5, 10**6, 8) if oracle.is_prime_trial(p))


def test_prime_batch_matches_singles_and_methods():
    rng = np.random.default_rng(5)
    ranges = []
    for _ in range(24):
        lo = int(10 ** rng.uniform(3, 11.5))
        ranges.append((lo, lo + int(rng.integers(1000, 3 * 10**6))))
    ranges.append((10**9, 10**9 + 8 * (1 << 24) + 1000))  # more than one pass
    a = [r[0] for r in ranges]
    b = [r[1] for r in ranges]
    with eis.Context(method=eis.Method.BABY) as cb:
        singles = [cb.eis_count_set(eis.EIS_SET_PRIME, x, y) for x, y in ranges]
    for method in (eis.Method.BABY, eis.Method.INFRA, eis.Method.AUTO):
        with eis.Context(method=method) as c:
            s, e = c.eis_count_batch_set(eis.EIS_SET_PRIME, a, b)
        assert [(int(x), int(y)) for x, y in zip(s, e)] == singles, method


def test_squarefree_set_is_eis_count_and_bad_set_rejected():
    with eis.Context() as c:
        assert c.eis_count_set(eis.EIS_SET_SQUAREFREE, 10**9, 10**9 + 10**6) == \
            c.eis_count(10**9, 10**9 + 10**6)
        with pytest.raises(eis.EisError) as ei:
            c.eis_count_set(7, 5, 100)
        assert ei.value.status == eis.Status.EINVAL
