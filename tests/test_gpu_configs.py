"""GPU test of the measurement-configuration driver: the small and the
method-comparison configurations run and report consistent numbers (the
driver itself refuses results where the two methods or the batched and
single calls disagree)."""
import sys

import pytest

import oracle
from paper_2507_06579_amd import configs, workloads

pytestmark = pytest.mark.gpu


def _say(msg):
    print(f"[gpu-configs] {msg}", flush=True)
    sys.stdout.flush()


def test_small_and_method_configs():
    _say("d1")
    d1 = configs.plain_latency(1)
    ref = oracle.classify_range(*workloads.SMALL, want_bits=False)
    assert (d1["pi_D"], d1["pi_E"]) == (ref["n_sqfree"], ref["n_eis"])
    _say("d2-like, 10^9 + 10^6")
    out = configs.methods_compared("d2", 10**9, 10**9 + 10**6, 1)
    assert out["identical_bits"]
    assert out["baby"]["giant_steps_per_s"] == 0 and out["infra"]["giant_steps_per_s"] > 0
    # the plain walk executes what it covers; the giant-step method covers more
    assert out["baby"]["executed_rho_per_s"] == pytest.approx(out["baby"]["covered_rho_per_s"], rel=1e-3)
    assert out["infra"]["executed_rho_per_s"] < out["infra"]["covered_rho_per_s"]
