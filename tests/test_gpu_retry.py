"""GPU tests of the retry round of the giant-step method.

Near 10^12 a few d's per 2^23 candidates fail a check of their giant steps:
a NUCOMP whose magnitudes pass 2^52 because one of the two ideals has a
small norm.  The retry round runs the first round's hand-offs again with
mu_1 four distinguished ideals later (other giant ideals), and the plain
walk takes only what the retry hands off again.  The bits must not change:
the whole window is compared with the oracle's golden (the sha256 of both
bitmaps, written by tests/golden/make_oracle_goldens.py from the oracle
alone) and with the plain walk's.
"""
import hashlib
import json
import os
import sys

import pytest

import paper_2507_06579_amd as eis

pytestmark = pytest.mark.gpu

# 2^23 candidates just below the largest supported bound
A, B = 10**12 - 2**26, 10**12

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "oracle_windows.json")


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
    assert retried > 0
    assert handed == 0  # the later mu_1 classifies every one of them here
    _say("plain walk on the same window")
    with eis.Context(method=eis.Method.BABY) as c:
        sq2, eb2, n_sq2, n_e2 = c.eis_classify(A, B)
    assert (n_sq, n_e) == (n_sq2, n_e2)
    assert bytes(sq) == bytes(sq2) and bytes(eb) == bytes(eb2)
    # both against the oracle's golden for this window
    with open(GOLDEN) as f:
        w = json.load(f)["windows"]["top_1e12"]
    assert (w["a"], w["b"]) == (A, B)
    nb = (w["n_cand"] + 7) // 8
    assert (n_sq, n_e) == (w["n_sqfree"], w["n_eis"])
    assert hashlib.sha256(bytes(sq[:nb])).hexdigest() == w["sha256_sqfree"]
    assert hashlib.sha256(bytes(eb[:nb])).hexdigest() == w["sha256_eis"]


def test_retry_round_is_timed_as_one_kernel():
    with eis.Context(method=eis.Method.INFRA, flags=eis.EIS_FLAG_KERNEL_TIMES) as c:
        c.eis_count(10**11 - 10**7, 10**11)
        st = c.eis_get_stats()
    k = eis.KERNELS.index("giant_retry")
    assert st["kernel_launches"][k] == 1
    assert st["kernel_launches"][eis.KERNELS.index("walk_giant")] == 1
    assert st["giant_retries"] == st["fallbacks"] == 0
