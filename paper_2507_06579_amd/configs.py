"""Measurement configurations beside the headline bench (one JSON line each).

  d1  plain walk on [5, 10^6 + 1): latency of one small classification;
  d2  [10^9, 10^9 + 10^7) with the plain walk and with the giant-step method
      on the same GPU: identical bitmaps required, times, executed rho steps
      per second, and "covered" steps per second (the plain walk's step
      count, i.e. the half-period lengths, divided by each method's time);
  d3  64 ranges of uneven height and width: one eis_count_batch call (a
      single pass per 2^24 candidates, replayed from a hipGraph) against 64
      eis_count calls, identical counts required;
  d4  the headline window [10^11 - 10^8, 10^11) with both methods, as d2.

The serving configuration (d5) is paper_2507_06579_amd.serve.  All work
runs in libeis.so; this module only times it.

  python -m paper_2507_06579_amd.configs [--reps 3] [--only d1,d2,d3,d4]
"""
from __future__ import annotations

import argparse
import json
import time

import numpy as np

from . import _lib as eis
from . import workloads


def _timed(fn, reps):
    """Best wall time of `reps` calls of fn (after one untimed call)."""
    out = fn()
    best = float("inf")
    for _ in range(reps):
        t = time.perf_counter()
        out = fn()
        best = min(best, time.perf_counter() - t)
    return out, best


def plain_latency(reps: int):
    a, b = workloads.SMALL
    with eis.Context(method=eis.Method.BABY) as c:
        (n_sq, n_e), dt = _timed(lambda: c.eis_count(a, b), reps)
    return {"config": "d1", "range": [a, b], "method": "baby", "pi_D": n_sq, "pi_E": n_e,
            "latency_ms": round(dt * 1e3, 3), "discriminants_per_s": round(n_sq / dt, 1)}


def methods_compared(name: str, a: int, b: int, reps: int):
    out = {"config": name, "range": [a, b]}
    bits = {}
    steps = {}
    for label, method in (("baby", eis.Method.BABY), ("infra", eis.Method.INFRA)):
        with eis.Context(method=method) as c:
            r = c.eis_classify(a, b)
            s0 = c.eis_get_stats()
            _, dt = _timed(lambda: c.eis_count(a, b), reps)
            s1 = c.eis_get_stats()
        calls = reps + 1  # _timed runs one untimed call first
        executed = (s1["baby_steps"] - s0["baby_steps"]) / calls
        giants = (s1["giant_steps"] - s0["giant_steps"]) / calls
        bits[label] = r
        steps[label] = executed
        out[label] = {"ms": round(dt * 1e3, 3), "discriminants_per_s": round(r[2] / dt, 1),
                      "executed_rho_per_s": round(executed / dt, 1),
                      "giant_steps_per_s": round(giants / dt, 1)}
    same = (np.array_equal(bits["baby"][0], bits["infra"][0])
            and np.array_equal(bits["baby"][1], bits["infra"][1])
            and bits["baby"][2:] == bits["infra"][2:])
    if not same:
        raise SystemExit(f"{name}: the two methods disagree")
    covered = steps["baby"]  # half-period lengths: what the plain walk executes
    for label in ("baby", "infra"):
        out[label]["covered_rho_per_s"] = round(covered / (out[label]["ms"] / 1e3), 1)
    out["pi_D"], out["pi_E"] = bits["baby"][2], bits["baby"][3]
    out["identical_bits"] = True
    return out


def batched_ranges(reps: int):
    ranges = workloads.batch_ranges()
    a = [x for x, _ in ranges]
    b = [y for _, y in ranges]
    with eis.Context() as c:
        c.eis_tune()
        (s_b, e_b), dt_batch = _timed(lambda: c.eis_count_batch(a, b), reps)
        singles, dt_single = _timed(lambda: [c.eis_count(x, y) for x, y in ranges], reps)
    if [int(x) for x in s_b] != [s for s, _ in singles] or [int(x) for x in e_b] != [e for _, e in singles]:
        raise SystemExit("d3: batched and single counts disagree")
    n_d = int(sum(s_b))
    return {"config": "d3", "ranges": len(ranges), "seed": workloads.BATCH_SEED,
            "members_of_D": n_d, "batched_ms": round(dt_batch * 1e3, 3),
            "singles_ms": round(dt_single * 1e3, 3),
            "batched_discriminants_per_s": round(n_d / dt_batch, 1),
            "singles_discriminants_per_s": round(n_d / dt_single, 1),
            "identical_counts": True}


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--reps", type=int, default=3)
    ap.add_argument("--only", default="d1,d2,d3,d4")
    args = ap.parse_args(argv)
    todo = set(args.only.split(","))
    if "d1" in todo:
        print(json.dumps(plain_latency(args.reps)), flush=True)
    if "d2" in todo:
        print(json.dumps(methods_compared("d2", *workloads.MID, args.reps)), flush=True)
    if "d3" in todo:
        print(json.dumps(batched_ranges(args.reps)), flush=True)
    if "d4" in todo:
        print(json.dumps(methods_compared("d4", *workloads.LARGE, 1)), flush=True)


if __name__ == "__main__":
    main()
