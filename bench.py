#!/usr/bin/env python3
"""Benchmark: Eisenstein-discriminant classification at d ~ 10^11 on one MI355X.

One step = one classification of the whole workload range (sieve, walks,
counts) through the C ABI, with device-resident outputs.  Prints ONE JSON
line (see the keys below).  The workload is the last 10^8-window below 10^11
(about 10.1 million members of D), whose Eisenstein count the paper prints
in Table 1 (3,345,503); the bench checks it.

  python bench.py [--gpus 1] [--steps K] [--warmup W] [--method auto|baby|infra]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "discriminants classified/sec and baby-steps/sec at d≈1e11; p99 query latency"
TABLE1_LARGE = 3345503

# VALU issue rate of MI355X: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz, one
# wave64 instruction per SIMD every 4 cycles = 39.3 T lane-slots/s.  (The
# published fp32 vector rate, 157.3 TFLOP/s, counts packed two-wide FMAs.)
PEAK_LANE_OPS = 256 * 64 * 2.4e9
# VALU issue slots per rho step of the walk kernels, counted in the gfx950
# code of the built loops (two steps per iteration, averaged) with the issue
# rules measured on the device (SQ_ACTIVE_INST_VALU / _VALU2 counters):
# v_rcp_f32 takes two slots, and v_fract_f32 / v_floor_f32 issue beside
# another VALU instruction of the same quad-cycle (no slot of their own).
# Plain walk: 11 VALU + rcp: the biased quotient (fma, mul, floor), the
# overshoot test, P' and Q' (fma, sub, fma), the residue (fract, fma) and
# two exit tests -> 11 + 2 (rcp) - 2 (floor, fract) = 11 slots.
VALU_SLOTS_PER_STEP = {"walk_plain": 11.0, "walk_handoff": 11.0}
# Window walk, per lane path like the giant walk's model: per rho step the
# same step (11), the distinguished-ideal test (mul, fract, cmp: 2) and the
# window-end tests (2 per pair: 1); per distinguished ideal
# appended (counted by the kernel, eis_stats.window_entries) the append: the
# selection of the pair's first distinguished ideal, LDS staging, count,
# residue sum and mu_1 bookkeeping (18 VALU) and an eighth of a chunk
# write-out (3 VALU).  The wave runs the append whenever any of its lanes
# appends; the lanes that do not append are not counted.
WINDOW_SLOTS = {"rho_steps": 14.0, "entries": 18.375}
# Giant-step walk: VALU issue slots per unit of its work, counted the same
# way in the gfx950 code of the built kernel (per-lane path; a branch that a
# lane does not take is not counted for it), the units being counted by the
# kernel itself (eis_stats giant_*):
#   composition, fixed part: the two ideal forms, NUCOMP on its common path
#     (gcd dividing s, partial Euclid with z != 0), the residue of gamma, the
#     set-up and final checks of the reduction, the kernel's bookkeeping: 330;
#   NUCOMP's gcd branch, when taken (H, l and their reductions mod H): 126;
#   Euclid step (extended or partial Euclid, two per loop iteration): 15;
#   reduction step after a composition (fp64, with its checks): 47;
#   walk step towards the next distinguished ideal (the step, the test): 11;
#   lookup of a distinguished ideal and its conjugate (hashes, first probe,
#     the extra step for the conjugate's key): 67.
GIANT_SLOTS = {"compositions": 330.0, "gcd_branches": 126.0, "euclid_steps": 15.0,
               "reduce_steps": 47.0, "walk_steps": 11.0, "lookups": 67.0}


# Device code whose HBM byte counts profiles/traffic.json records; the
# record is used only while these files are unchanged.
DEVICE_SOURCES = ["eis_kernels.hip", "eis_infra.hip", "eis_walk.h", "eis_giant.h",
                  "eis_internal.h"]


def device_sources_sha256() -> str:
    import hashlib
    h = hashlib.sha256()
    for name in DEVICE_SOURCES:
        with open(os.path.join(ROOT, "paper_2507_06579_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def measured_traffic(kernel: str, workload: str):
    """HBM bytes per launch of `kernel` on `workload` from the counter runs
    recorded in profiles/traffic.json (FETCH_SIZE and WRITE_SIZE, each scaled
    by the same counter's reading for a copy of known size), or None when
    there is no record or the device code has changed since."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        doc = json.load(f)
    ent = doc.get(kernel, {}).get(workload)
    if not ent or ent.get("device_sources_sha256") != device_sources_sha256():
        return None
    return int(ent["hbm_bytes_per_launch"])


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def cpu_baseline(a: int, b: int, target_s: float = 15.0):
    """The oracle (full-period walk, mod-2 mode) on a bounded random sample of
    the members of D in [a, b), timed on this host's cores."""
    import numpy as np
    import oracle
    from paper_2507_06579_amd import workloads
    bits, _ = oracle.sqfree_range(a, b)
    n = oracle.num_candidates(a, b)
    d0 = oracle.first_candidate(a)
    idx = np.flatnonzero(np.unpackbits(bits, bitorder="little")[:n])
    cores = os.cpu_count() or 1
    rng_idx = workloads.sample_indices(idx.size, idx.size, seed=7)
    members = d0 + 8 * idx[rng_idx].astype(np.uint64)
    # calibrate on a small batch, then size the sample for about target_s
    k0 = min(4 * cores, members.size)
    t = time.perf_counter()
    oracle.classify_list(members[:k0], nthreads=cores)
    dt0 = max(time.perf_counter() - t, 1e-3)
    k = int(min(members.size - k0, max(cores, k0 * target_s / dt0)))
    sample = members[k0:k0 + k]
    t = time.perf_counter()
    _, steps = oracle.classify_list(sample, nthreads=cores)
    dt = time.perf_counter() - t
    # one thread, on a sample sized for about 3 s
    k1 = max(1, min(sample.size, int(sample.size * 3.0 / (dt * cores))))
    t = time.perf_counter()
    oracle.classify_list(sample[:k1], nthreads=1)
    rate1 = k1 / (time.perf_counter() - t)
    return {"value": round(sample.size / dt, 2), "unit": "discriminants/s", "cores": cores,
            "kind": "oracle",
            "sample": f"{sample.size} random members of D in [{a}, {b}), full-period walk "
                      f"({steps} rho steps, {dt:.1f} s on {cores} threads of {cpu_model()}); "
                      f"one thread: {rate1:.1f} discriminants/s on {k1} of them"}


def cpu_model() -> str:
    """The host CPU's model name (from /proc/cpuinfo), or 'unknown CPU'."""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown CPU"


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--method", default="auto", choices=["auto", "baby", "infra"])
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="run one elementwise copy of this many MiB before the workload "
                         "(the reference kernel for scaling HBM byte counters)")
    ap.add_argument("--window-scale", type=float, default=0.0,
                    help="giant-step window scale (0: tuned or default)")
    ap.add_argument("--no-tune", action="store_true",
                    help="auto method without running the autotuner first")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-serving", action="store_true")
    ap.add_argument("--serve-rate", type=float, default=100.0)
    ap.add_argument("--serve-n", type=int, default=300)
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only: the per-d walks "
                                   "are independent, so a range would shard into blocks of "
                                   "equal estimated cost, one per GPU, whose two counts are "
                                   "summed; that sharding is not run here"}), flush=True)
        sys.exit(2)

    import torch
    import paper_2507_06579_amd as eis
    from paper_2507_06579_amd import workloads

    a, b = workloads.LARGE
    method = {"auto": eis.Method.AUTO, "baby": eis.Method.BABY, "infra": eis.Method.INFRA}[args.method]
    n = eis.eis_num_candidates(a, b)
    nb = (n + 7) // 8
    dev = torch.device("cuda:0")
    sq = torch.zeros(nb, dtype=torch.uint8, device=dev)
    eb = torch.zeros(nb, dtype=torch.uint8, device=dev)
    counts = torch.zeros(2, dtype=torch.int64, device=dev)
    ctx = eis.Context(device=0, method=method, flags=eis.EIS_FLAG_KERNEL_TIMES,
                      window_scale=args.window_scale)
    if method == eis.Method.AUTO and not args.no_tune:
        t = time.perf_counter()
        ctx.eis_tune()
        log(f"autotuner: {time.perf_counter() - t:.1f} s")
    chosen, wscale = ctx.eis_tuned_choice(a)
    log(f"method at d={a}: {chosen.name}, window scale {wscale}")

    def step():
        ctx.eis_classify_async(a, b, sq.data_ptr(), eb.data_ptr(), counts.data_ptr(), 0)

    if args.copy_probe_mib:
        src = torch.ones(args.copy_probe_mib << 18, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        torch.mul(src, 1.0, out=dst)
        torch.cuda.synchronize()
        log(f"copy probe: {args.copy_probe_mib} MiB read, {args.copy_probe_mib} MiB written")
        del src, dst
    log(f"workload [{a}, {b}) candidates={n} method={args.method}")
    for i in range(args.warmup):
        step()
        rc = ctx.eis_last_error()
        if rc != 0:
            raise SystemExit(f"warmup step failed: {eis.eis_strerror(rc)}")
        log(f"warmup {i + 1}/{args.warmup} done")
    torch.cuda.synchronize()
    base = ctx.eis_get_stats()
    walk_ms = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        step()
        rc = ctx.eis_last_error()  # synchronises the context stream
        if rc != 0:
            raise SystemExit(f"step failed: {eis.eis_strerror(rc)}")
        walk_ms.append(ctx.eis_get_stats()["last_walk_ms"])
        log(f"step {i + 1}/{args.steps} walk {walk_ms[-1]:.1f} ms")
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    st = ctx.eis_get_stats()
    n_sq, n_e = counts.cpu().tolist()
    if n_e != TABLE1_LARGE:
        raise SystemExit(f"pi_E of the window is {n_e}, Table 1 says {TABLE1_LARGE}")
    kms = [x - y for x, y in zip(st["kernel_ms"], base["kernel_ms"])]
    kl = [x - y for x, y in zip(st["kernel_launches"], base["kernel_launches"])]
    ks = [x - y for x, y in zip(st["kernel_steps"], base["kernel_steps"])]
    discs = st["discriminants"] - base["discriminants"]
    baby = st["baby_steps"] - base["baby_steps"]
    giant = st["giant_steps"] - base["giant_steps"]
    value = discs / elapsed
    ms_per_step = 1e3 * elapsed / args.steps
    kernels = {}
    for k, name in enumerate(eis.KERNELS):
        if kl[k]:
            kernels[name] = {"ms_per_step": round(kms[k] / args.steps, 3),
                             "launches_per_step": kl[k] / args.steps,
                             "rho_steps_per_step": ks[k] // args.steps}
    # dominant kernel: the walk kernel with the largest share of the step
    # (the other kernels of a pass take a few percent of it)
    walks = list(VALU_SLOTS_PER_STEP) + ["walk_window", "walk_giant"]

    def slot_model(name):
        """(VALU slots, units of work, unit name, model details) of the
        timed launches of a walk kernel."""
        k = eis.KERNELS.index(name)
        if name == "walk_window":
            work = {"rho_steps": ks[k], "entries": st["window_entries"] - base["window_entries"]}
            slots = sum(WINDOW_SLOTS[key] * v for key, v in work.items())
            return (slots, ks[k], "rho step",
                    {"slots": WINDOW_SLOTS,
                     "work_per_launch": {key: int(v / kl[k]) for key, v in work.items()}})
        if name != "walk_giant":
            return VALU_SLOTS_PER_STEP[name] * ks[k], ks[k], "rho step", None
        work = {key: st["giant_" + key] - base["giant_" + key]
                for key in ("compositions", "gcd_branches", "euclid_steps", "reduce_steps",
                            "lookups")}
        work["walk_steps"] = ks[k]
        slots = sum(GIANT_SLOTS[key] * v for key, v in work.items())
        fill = {}
        for ph in ("compose", "walk"):
            nph = st[f"giant_{ph}_phases"] - base[f"giant_{ph}_phases"]
            nln = st[f"giant_{ph}_lanes"] - base[f"giant_{ph}_lanes"]
            fill[ph] = {"phases_per_launch": int(nph / kl[k]),
                        "busy_lanes_per_phase": round(nln / max(1, nph), 2)}
        return (slots, work["compositions"],
                "giant step (composition, reduction, walk to a distinguished ideal, lookup)",
                {"slots": GIANT_SLOTS,
                 "work_per_launch": {key: int(v / kl[k]) for key, v in work.items()},
                 "phase_fill": fill})

    dom = max(walks, key=lambda name: kms[eis.KERNELS.index(name)])
    kd = eis.KERNELS.index(dom)
    avg_launch_s = kms[kd] / kl[kd] / 1e3
    slots, units, unit_of_work, model = slot_model(dom)
    achieved = slots / kl[kd] / avg_launch_s
    kernel_name = {"walk_plain": "k_walk_baby", "walk_handoff": "k_walk_baby",
                   "walk_window": "k_walk_window", "walk_giant": "k_walk_giant"}[dom]
    roofline = {"bound": "alu", "achieved": round(achieved / 1e12, 3),
                "peak": round(PEAK_LANE_OPS / 1e12, 3), "unit": "T VALU lane-slots/s",
                "frac": round(achieved / PEAK_LANE_OPS, 4),
                "traffic": None,
                "kernel": kernel_name,
                "ops_per_unit": round(slots / max(1, units), 1), "unit_of_work": unit_of_work,
                "units_per_launch": int(units / kl[kd]),
                "avg_launch_ms": round(avg_launch_s * 1e3, 3),
                "share_of_step_time": round(kms[kd] / (1e3 * elapsed), 3)}
    if model:
        roofline["model"] = model
    # the other walk kernels of the step, on the same model
    others = {}
    for name in walks:
        k = eis.KERNELS.index(name)
        if name == dom or not kl[k] or not ks[k]:
            continue
        sl, un, uw, md = slot_model(name)
        a_k = sl / (kms[k] / 1e3)
        others[name] = {"achieved": round(a_k / 1e12, 3), "frac": round(a_k / PEAK_LANE_OPS, 4),
                        "ms_per_step": round(kms[k] / args.steps, 3),
                        "avg_launch_ms": round(kms[k] / kl[k], 3),
                        "ops_per_unit": round(sl / max(1, un), 1), "unit_of_work": uw,
                        "units_per_launch": int(un / kl[k])}
        if md:
            others[name]["model"] = md
    roofline["traffic"] = measured_traffic(roofline["kernel"], f"large:{chosen.name.lower()}")
    out = {
        "metric": METRIC,
        "value": round(value, 1),
        "unit": "discriminants/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int32/fp32-exact",
        "data": "synthetic: the integer range itself (no dataset)",
        "config": {"workload": f"large height: all d = 5 mod 8 in [{a}, {b})",
                   "candidates": n, "members_of_D": n_sq, "pi_E": n_e,
                   "method": args.method, "chosen_method": chosen.name.lower(),
                   "window_scale": wscale},
        "baby_steps_per_s": round(baby / elapsed, 1),
        "fallbacks_per_step": (st["fallbacks"] - base["fallbacks"]) // args.steps,
        "giant_steps_per_s": round(giant / elapsed, 1),
        "kernels": kernels,
        "roofline": roofline,
        "roofline_other_walks": others,
    }
    if not args.no_serving:
        from paper_2507_06579_amd import serve
        log(f"serving: {args.serve_n} requests, Poisson at {args.serve_rate} req/s")
        reqs = workloads.serve_requests(args.serve_n, args.serve_rate)
        with eis.Context(device=0, serve_slots=256) as sctx:
            res = serve.run_open_loop(sctx, reqs)
        srv = serve.summarize(res, reqs)
        srv["rate_req_s"] = args.serve_rate
        srv["workload"] = ("range counts [a, a+w), a log-uniform in [1e6, 1e11], "
                           "w log-uniform in [1e3, 1e7]")
        out["p99_query_latency_ms"] = srv["p99_ms"]
        out["serving"] = srv
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle on a bounded sample)")
        out["cpu_baseline"] = cpu_baseline(a, b)
    ctx.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
