"""Open-loop serving driver: range-count queries through eis_submit / eis_wait.

Arrivals follow a precomputed Poisson schedule (so a slow server does not
slow the offered load: no coordinated omission); one thread submits on
schedule, a pool of waiter threads collects results.  Latency is submit to
result.  All work happens in libeis.so; this module only times it.

  python -m paper_2507_06579_amd.serve --rates 10,30,100,300,1000 --n 2000
"""
from __future__ import annotations

import argparse
import json
import queue
import threading
import time

import numpy as np

from . import _lib as eis
from . import workloads


def run_open_loop(ctx, requests, n_waiters: int = 32, timeout_s: float = 600.0):
    """Serve `requests` = [(t_arrival_s, a, b), ...].

    Returns dict(latency_ms array in submission order, counts list, wall_s,
    rejected) -- a request refused with EIS_EBUSY is retried after a short
    back-off, and its latency still starts at its scheduled arrival."""
    n = len(requests)
    lat = np.zeros(n)
    counts = [None] * n
    pending = queue.Queue()
    errors = []

    def waiter():
        while True:
            item = pending.get()
            if item is None:
                return
            k, ticket, t_sched = item
            try:
                counts[k] = ctx.eis_wait(ticket, int(timeout_s * 1e6))
            except eis.EisError as e:  # noqa: PERF203
                errors.append((k, e))
            lat[k] = (time.perf_counter() - t_sched) * 1e3

    ths = [threading.Thread(target=waiter, daemon=True) for _ in range(n_waiters)]
    for th in ths:
        th.start()
    rejected = 0
    t0 = time.perf_counter()
    for k, (t_arr, a, b) in enumerate(requests):
        t_sched = t0 + t_arr
        now = time.perf_counter()
        if t_sched > now:
            time.sleep(t_sched - now)
        while True:
            try:
                ticket = ctx.eis_submit(a, b)
                break
            except eis.EisError as e:
                if e.status != eis.Status.EBUSY:
                    raise
                rejected += 1
                time.sleep(0.0005)
        pending.put((k, ticket, t_sched))
    for _ in ths:
        pending.put(None)
    for th in ths:
        th.join()
    wall = time.perf_counter() - t0
    if errors:
        raise RuntimeError(f"{len(errors)} requests failed, first: {errors[0]}")
    return {"latency_ms": lat, "counts": counts, "wall_s": wall, "rejected": rejected}


def summarize(res, requests):
    lat = res["latency_ms"]
    discs = sum(c[0] for c in res["counts"])
    return {
        "requests": len(requests),
        "p50_ms": round(float(np.percentile(lat, 50)), 3),
        "p99_ms": round(float(np.percentile(lat, 99)), 3),
        "max_ms": round(float(lat.max()), 3),
        "throughput_req_s": round(len(requests) / res["wall_s"], 2),
        "discriminants_per_s": round(discs / res["wall_s"], 1),
        "busy_retries": res["rejected"],
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--rates", default="10,30,100,300,1000")
    ap.add_argument("--n", type=int, default=2000, help="requests per rate")
    ap.add_argument("--max-seconds", type=float, default=60.0,
                    help="cap on the schedule length per rate")
    ap.add_argument("--slots", type=int, default=256)
    args = ap.parse_args()
    ctx = eis.Context(serve_slots=args.slots)
    for rate in [float(r) for r in args.rates.split(",")]:
        n = min(args.n, max(1, int(rate * args.max_seconds)))
        reqs = workloads.serve_requests(n, rate)
        res = run_open_loop(ctx, reqs)
        out = {"rate_req_s": rate, "seed": workloads.SERVE_SEED}
        out.update(summarize(res, reqs))
        print(json.dumps(out), flush=True)
    ctx.close()


if __name__ == "__main__":
    main()
