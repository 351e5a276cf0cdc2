"""GPU tests of the paper-scale sweep driver: pi_E(10^8) is the sum of the
first Table 1 window (3,259,668, pinned for the oracle too), and a sweep
resumed from a partial checkpoint gives the same counts."""
import json
import sys

import pytest

import oracle
from paper_2507_06579_amd import sweep

pytestmark = pytest.mark.gpu

TABLE1_FIRST = 3259668  # Table 1, [0, 10^8], sum of the Total column


def _say(msg):
    print(f"[gpu-sweep] {msg}", flush=True)
    sys.stdout.flush()


def test_sweep_to_1e8_and_resume(tmp_path):
    cp = str(tmp_path / "sweep.json")
    _say("sweep to 1e8")
    full = sweep.run(10**8, 10**9, cp, per_call=3, log=_say)
    assert full["pi_E"] == TABLE1_FIRST
    # a fresh run classifies every member of D once
    assert full["work"]["discriminants"] == full["pi_D"]
    pw = {p["x"]: p for p in full["powers_of_ten"]}
    for k in range(1, 7):
        ref = oracle.classify_range(0, 10**k, want_bits=False)
        assert (pw[10**k]["pi_D"], pw[10**k]["pi_E"]) == (ref["n_sqfree"], ref["n_eis"]), k
    # drop the last two segments from the checkpoint and resume
    doc = json.load(open(cp))
    doc["segments"] = doc["segments"][:-2]
    json.dump(doc, open(cp, "w"))
    _say("resume")
    again = sweep.run(10**8, 10**9, cp, per_call=3, log=_say)
    assert (again["pi_D"], again["pi_E"]) == (full["pi_D"], full["pi_E"])
    assert again["density"] == full["density"]


def test_prime_sweep_matches_oracle_at_powers_of_ten(tmp_path):
    cp = str(tmp_path / "primes.json")
    _say("prime sweep to 1e7")
    out = sweep.run(10**7, 10**9, cp, per_call=4, log=_say, which="prime")
    assert out["set"] == "prime"
    pw = {p["x"]: p for p in out["powers_of_ten"]}
    for k in range(1, 8):
        n_p, n_e = oracle.classify_primes(0, 10**k)
        assert (pw[10**k]["pi_DP"], pw[10**k]["pi_EP"]) == (n_p, n_e), k
    # pi(10^7) = 664,579 primes, of which about a quarter are 5 mod 8
    assert abs(out["pi_DP"] - 664579 / 4) < 300
    with pytest.raises(SystemExit):
        sweep.run(10**7, 10**9, cp, per_call=4, log=_say, which="squarefree")
