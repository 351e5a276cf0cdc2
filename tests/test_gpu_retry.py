"""GPU tests of the retry round of the giant-step method.

Near 10^12 a few d's per 2^23 candidates fail a check of their giant steps:
a NUCOMP whose magnitudes pass 2^52 because one of the two ideals has a
small norm.  The retry round runs the first round's hand-offs again with
mu_1 four distinguished ideals later (other giant ideals), and the plain
walk takes only what the retry hands off again.  The bits must not change:
they are compared with the plain walk's over the whole window (the plain
walk is pinned to the oracle by the parity tests), and the d's that a CPU
replay of the giant-step arithmetic finds failing in this window are
checked against the oracle one by one.
"""
import sys

import numpy as np
import pytest

import oracle
import paper_2507_06579_amd as eis

pytestmark = pytest.mark.gpu

# 2^23 candidates just below the largest supported bound
A, B = 10**12 - 2**26, 10**12

# members of D in [A, B) whose first giant-step attempt at window scale 2.0
# fails the 2^52 check (found by replaying the device arithmetic on the CPU)
FIRST_ROUND_FAILURES = [999938662941, 999940370501, 999941547781, 999943250797]


def _say(msg):
    print(f"[gpu-retry] {msg}", flush=True)
    sys.stdout.flush()


def test_retry_round_keeps_bits_and_ends_the_handoffs():
    _say(f"giant-step method on [{A}, {B})")
    with eis.Context(method=eis.Method.INFRA, window_scale=2.0) as c:
        s0 = c.eis_get_stats()
        sq, eb, n_sq, n_e = c.eis_classify(A, B)
        s1 = c.eis_get_stats()
    retried = s1["giant_retries"] - s0["giant_retries"]
    handed = s1["fallbacks"] - s0["fallbacks"]
    _say(f"retried {retried}, handed to the plain walk {handed}")
    assert retried >= len(FIRST_ROUND_FAILURES)
    assert handed == 0  # the later mu_1 classifies every one of them here
    _say("plain walk on the same window")
    with eis.Context(method=eis.Method.BABY) as c:
        sq2, eb2, n_sq2, n_e2 = c.eis_classify(A, B)
    assert (n_sq, n_e) == (n_sq2, n_e2)
    assert bytes(sq) == bytes(sq2) and bytes(eb) == bytes(eb2)
    # the retried d's against the oracle
    first = oracle.first_candidate(A)
    bits = np.unpackbits(np.frombuffer(bytes(eb), dtype=np.uint8), bitorder="little")
    flags, _ = oracle.classify_list(FIRST_ROUND_FAILURES)
    for d, f in zip(FIRST_ROUND_FAILURES, flags):
        assert oracle.in_D_trial(d)
        assert bits[(d - first) // 8] == f, d


def test_retry_round_is_timed_as_one_kernel():
    with eis.Context(method=eis.Method.INFRA, flags=eis.EIS_FLAG_KERNEL_TIMES) as c:
        c.eis_count(10**11 - 10**7, 10**11)
        st = c.eis_get_stats()
    k = eis.KERNELS.index("giant_retry")
    assert st["kernel_launches"][k] == 1
    assert st["kernel_launches"][eis.KERNELS.index("walk_giant")] == 1
    assert st["giant_retries"] == st["fallbacks"] == 0
