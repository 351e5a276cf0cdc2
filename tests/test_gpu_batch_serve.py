"""GPU tests of the batched call and of serving.

Counts are integers: every comparison is exact.  Each batched or served
result must equal the result of the same range computed alone (which the
single-range parity tests pin to the oracle), and small ranges are also
checked against the oracle directly.
"""
import sys
import threading
import time

import numpy as np
import pytest

import oracle
import paper_2507_06579_amd as eis
from paper_2507_06579_amd import workloads

pytestmark = pytest.mark.gpu


def _say(msg):
    print(f"[gpu-batch] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ranges64():
    return workloads.batch_ranges(64)


@pytest.fixture(scope="module")
def singles(ranges64):
    with eis.Context(method=eis.Method.BABY) as c:
        _say("64 ranges one by one (plain walk)")
        return [c.eis_count(a, b) for a, b in ranges64]


def test_batch_matches_single_ranges(ranges64, singles):
    a = [r[0] for r in ranges64]
    b = [r[1] for r in ranges64]
    with eis.Context(method=eis.Method.AUTO) as c:
        _say("batched, auto method, graph replays")
        for rep in range(3):
            s, e = c.eis_count_batch(a, b)
            assert [(int(x), int(y)) for x, y in zip(s, e)] == singles, rep
            # eager work between the replays
            assert c.eis_count(*ranges64[rep]) == singles[rep]


def test_batch_without_graphs_and_methods(ranges64, singles):
    a = [r[0] for r in ranges64]
    b = [r[1] for r in ranges64]
    for method in (eis.Method.BABY, eis.Method.INFRA):
        with eis.Context(method=method, flags=eis.EIS_FLAG_NO_GRAPHS) as c:
            _say(f"batched, {eis.Method(method).name}, no graphs")
            s, e = c.eis_count_batch(a, b)
            assert [(int(x), int(y)) for x, y in zip(s, e)] == singles


def test_batch_small_ranges_against_oracle():
    rng = np.random.default_rng(99)
    ranges = []
    for _ in range(40):
        lo = int(10 ** rng.uniform(1, 8))
        ranges.append((lo, lo + int(rng.integers(0, 20000))))
    ranges += [(5, 6), (6, 13), (0, 0), (100, 50)]
    with eis.Context() as c:
        s, e = c.eis_count_batch([r[0] for r in ranges], [r[1] for r in ranges])
    for (a, b), x, y in zip(ranges, s, e):
        r = oracle.classify_range(a, b, want_bits=False) if a < b else {"n_sqfree": 0, "n_eis": 0}
        assert (int(x), int(y)) == (r["n_sqfree"], r["n_eis"]), (a, b)


def test_batch_many_pieces():
    # more pieces than fit one pass: both limits of a pass are exercised
    ranges = [(10**7 + 1000 * k, 10**7 + 1000 * k + 997) for k in range(300)]
    ranges.append((2 * 10**9, 2 * 10**9 + 8 * (1 << 24) + 40))
    with eis.Context() as c:
        s, e = c.eis_count_batch([r[0] for r in ranges], [r[1] for r in ranges])
        for k in (0, 150, 299, 300):
            assert (int(s[k]), int(e[k])) == c.eis_count(*ranges[k])
    for k in (0, 299):
        assert int(s[k]) == oracle.mobius_count(*ranges[k])


def test_serving_results_equal_alone():
    reqs = workloads.serve_requests(60, rate=200.0)
    with eis.Context(method=eis.Method.BABY) as c0:
        alone = [c0.eis_count(a, b) for _, a, b in reqs]
    with eis.Context(serve_slots=64) as c:
        _say("serving 60 requests, open loop at 200 req/s")
        tickets = []
        t0 = time.perf_counter()
        for t_arr, a, b in reqs:
            now = time.perf_counter() - t0
            if t_arr > now:
                time.sleep(t_arr - now)
            tickets.append(c.eis_submit(a, b))
        got = [c.eis_wait(t, 30_000_000) for t in tickets]
        st = c.eis_get_stats()
    assert got == alone
    assert st["requests_done"] == len(reqs)


def test_serving_admission_and_cancel():
    with eis.Context(serve_slots=2) as c:
        # two requests of several passes each fill both slots
        b1 = c.eis_submit(10**11 - 8 * 10**7, 10**11)
        b2 = c.eis_submit(10**11 - 16 * 10**7, 10**11 - 8 * 10**7)
        with pytest.raises(eis.EisError) as ei:
            c.eis_submit(5, 1000)
        assert ei.value.status == eis.Status.EBUSY
        c.eis_cancel(b1)
        c.eis_cancel(b2)
        for t in (b1, b2):
            rc, _, _ = c.eis_wait_status(t, 30_000_000)
            assert rc == eis.Status.ECANCELED
        # slots are free again
        t = c.eis_submit(5, 1000)
        assert c.eis_wait(t, 30_000_000) == (oracle.mobius_count(5, 1000),
                                            oracle.classify_range(5, 1000)["n_eis"])
        with pytest.raises(eis.EisError):
            c.eis_wait(123456789, 0)


def test_serving_concurrent_waiters():
    with eis.Context(serve_slots=16) as c:
        small = [c.eis_submit(10**6 + 100 * k, 10**6 + 100 * k + 5000) for k in range(8)]
        results = {}

        def waiter(t):
            results[t] = c.eis_wait(t, 30_000_000)

        ths = [threading.Thread(target=waiter, args=(t,)) for t in small]
        for th in ths:
            th.start()
        for th in ths:
            th.join()
        for k, t in enumerate(small):
            a = 10**6 + 100 * k
            ref = oracle.classify_range(a, a + 5000, want_bits=False)
            assert results[t] == (ref["n_sqfree"], ref["n_eis"])
        # two waiters on one ticket: one retires it with the result, the
        # other returns EINVAL (unknown ticket) instead of waiting on
        t = c.eis_submit(10**9, 10**9 + 10**6)
        rcs = []

        def waiter2():
            rcs.append(c.eis_wait_status(t, 30_000_000))

        ths = [threading.Thread(target=waiter2) for _ in range(2)]
        for th in ths:
            th.start()
        for th in ths:
            th.join()
        codes = sorted(int(r[0]) for r in rcs)
        assert codes == sorted([int(eis.Status.OK), int(eis.Status.EINVAL)]), rcs
        ok = [r for r in rcs if r[0] == eis.Status.OK][0]
        assert (ok[1], ok[2]) == c.eis_count(10**9, 10**9 + 10**6)
        # a timed-out wait leaves the ticket pending
        t = c.eis_submit(10**10, 10**10 + 10**6)
        rc, s, e = c.eis_wait_status(t, 0)
        assert rc in (eis.Status.ETIMEDOUT, eis.Status.OK)
        if rc == eis.Status.ETIMEDOUT:
            s, e = c.eis_wait(t, 30_000_000)
        assert (s, e) == c.eis_count(10**10, 10**10 + 10**6)


def test_serving_admission_by_device_memory():
    """A small memory budget: a request whose giant-step scratch cannot fit
    even alone is refused with ENOMEM, requests that fit are admitted while
    the reservations of the admitted ones leave room (EBUSY otherwise), the
    plain walk's heights need no reservation, and every admitted result
    equals the oracle's."""
    budget = 200 * 2**20 + 300 * 2**20  # about the fixed buffers + 300 MiB
    with eis.Context(mem_budget_bytes=budget, serve_slots=256) as c:
        t_plain = c.eis_submit(10**6, 10**6 + 80000)  # plain walk: no reservation
        st = c.eis_get_stats()
        sb = st["serve_bytes_budget"]
        _say(f"serving budget {sb} bytes")
        assert 0 < sb < budget
        # 2^20 candidates near 10^11 need about 2 GB of dictionaries
        with pytest.raises(eis.EisError) as ei:
            c.eis_submit(10**11 - 8 * 2**20, 10**11)
        assert ei.value.status == eis.Status.ENOMEM
        # 40,000 candidates near 10^11 need about 76 MB each: a few at a time
        ranges = [(10**11 - 8 * 40000 * (k + 1), 10**11 - 8 * 40000 * k) for k in range(24)]
        admitted, busy = [], 0
        for a, b in ranges:
            try:
                admitted.append((c.eis_submit(a, b), a, b))
            except eis.EisError as e:
                assert e.status == eis.Status.EBUSY
                busy += 1
            assert c.eis_get_stats()["serve_bytes_reserved"] <= sb
        _say(f"admitted {len(admitted)}, refused {busy} (memory)")
        assert busy > 0 and len(admitted) >= 2
        got = [(c.eis_wait(t, 60_000_000), a, b) for t, a, b in admitted]
        assert c.eis_wait(t_plain, 60_000_000) == (
            oracle.mobius_count(10**6, 10**6 + 80000),
            oracle.classify_range(10**6, 10**6 + 80000, want_bits=False)["n_eis"])
        assert c.eis_get_stats()["serve_bytes_reserved"] == 0
        for (res, a, b) in got[:3]:
            ref = oracle.classify_range(a, b, want_bits=False)
            assert res == (ref["n_sqfree"], ref["n_eis"]), (a, b)
        # memory freed: a refused range is admitted now
        a, b = ranges[-1]
        t = c.eis_submit(a, b)
        assert c.eis_wait(t, 60_000_000) == c.eis_count(a, b)
