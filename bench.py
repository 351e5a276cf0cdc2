#!/usr/bin/env python3
"""Benchmark: Eisenstein-discriminant classification at d ~ 10^11 on one MI355X.

One step = one classification of the whole workload range (sieve, walks,
counts) through the C ABI, with device-resident outputs.  Prints ONE JSON
line (see the keys below).  The workload is the last 10^8-window below 10^11
(about 10.1 million members of D), whose Eisenstein count the paper prints
in Table 1 (3,345,503); the bench checks it.

The same line carries, under "configs", the other measurement
configurations, each with its time, discriminants/s, the walk kernels'
roofline fractions (VALU issue slots of their counted work over their
event-timed duration) and the oracle's rate on a bounded sample of the same
workload: d1 the plain walk on [5, 10^6]; d2 [10^9, 10^9 + 10^7) with both
methods (identical bitmaps required); d3 the 64 seeded uneven ranges, one
batched call against 64 single calls; d5 the seeded Poisson request stream
served at 10 to 10^4 requests/s, past saturation (p50/p99 latency,
throughput).  The headline roofline comes from the headline steps alone;
its `traffic` (HBM bytes per launch of the dominant kernel) is measured in
the same run: the headline step once more in two child processes under
rocprofv3 --pmc (FETCH_SIZE, then WRITE_SIZE), with this run's tuned choices
and a 1 GiB copy to scale the counters (profiles/traffic.json is the
fallback when rocprofv3 is missing, valid only for the recorded sources).

  python bench.py [--gpus 1] [--steps K] [--warmup W] [--method auto|baby|infra]
                  [--no-configs] [--no-serving] [--no-cpu-baseline] [--no-tune]
                  [--tune-cache PATH] [--no-traffic]
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
# Plain walk: 10 VALU + rcp: the biased quotient (fma, mul, floor), P' and Q'
# (fma, sub, fma), the residue (fract, fma) and two exit tests -> 10 + 2
# (rcp) - 2 (floor, fract) = 10 slots.  These counts are for passes whose d's
# are all at most 1.45e11 (every workload here): their walks leave the
# quotient's overshoot test out; above that height a step has one more slot.
VALU_SLOTS_PER_STEP = {"walk_plain": 10.0, "walk_handoff": 10.0}
# Window walk, per lane path like the giant walk's model, counted in the
# gfx950 code of the built kernel with the same issue rules: per rho step the
# step with its two half-period compares (10), the distinguished-ideal test
# (mul, fract, cmp: 2) and half of the two per-pair window tests (mu_1
# staged, window end: 1); per distinguished ideal appended (counted by the
# kernel, eis_stats.window_entries) the append: the selection of the pair's
# first distinguished ideal, its residue sum and step, LDS staging and count
# (15) and a quarter of a four-entry chunk write-out (3).  The wave runs the append
# whenever any of its lanes appends; the lanes that do not append are not
# counted.  mu_1's bookkeeping (once per window) and a window's end (written
# at the wave's next pause) are not counted.
WINDOW_SLOTS = {"rho_steps": 13.0, "entries": 15.75}
# Giant-step walk: VALU issue slots per unit of its work, counted the same
# way in the gfx950 code of the built kernel (per-lane path; a branch that a
# lane does not take is not counted for it), the units being counted by the
# kernel itself (eis_stats giant_*):
#   composition, fixed part: the two ideal forms, NUCOMP on its common path
#     (gcd dividing s, partial Euclid with z != 0), the residue of gamma, the
#     set-up and final checks of the reduction, the kernel's bookkeeping: 330;
#   NUCOMP's gcd branch, when taken (the second Bezout cofactor, H, l and
#     their reductions mod H): 136;
#   extended Euclid step (nearest-integer quotients, two per loop iteration
#     of 18: the iteration count's copy 1, per step the reciprocal 2, the
#     quotient, remainder, cofactor, tests and selects 6; v_rndne_f32
#     counted like v_floor_f32): 9;
#   partial Euclid step (floor quotients, whose estimate needs no
#     correction for the norms of d <= 10^12; two per loop iteration of 21,
#     the iteration count's copy included): 10.5;
#   reduction step after a composition (fp64, with its checks and the loop
#     test, two steps per iteration on swapping registers): 45;
#   walk step towards the next distinguished ideal (the step, the test): 10;
#   lookup of a distinguished ideal and its conjugate (the extra step for
#     the conjugate's key, two hashes, home groups, fingerprints and group
#     addresses: 43; the byte-parallel fingerprint match of two 8-slot
#     groups, the list addresses and the tests on a lane's path when no slot
#     matches: 69): 112.
GIANT_SLOTS = {"compositions": 330.0, "gcd_branches": 136.0, "xgcd_steps": 9.0,
               "partial_euclid_steps": 10.5, "reduce_steps": 45.0, "walk_steps": 10.0,
               "lookups": 112.0}


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


TRAFFIC_KERNELS = ["k_walk_giant", "k_walk_window", "k_build_tables", "k_giant_square"]


def traffic_from_counters(fetch_dir: str, write_dir: str, probe_mib: int):
    """HBM bytes per launch of each kernel in TRAFFIC_KERNELS from the output
    folders of two rocprofv3 --pmc runs of this bench (one step,
    --copy-probe-mib probe_mib): FETCH_SIZE and WRITE_SIZE (KiB per dispatch)
    of the kernel's last dispatch, each scaled by what the same counter reads
    for the copy probe (probe_mib MiB read and written).  Returns
    ({kernel: (fetch_kib, write_kib, bytes)}, probe record); host only."""
    import csv
    import glob

    def read(d, counter):
        files = glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True)
        if not files:
            raise RuntimeError(f"no counter_collection.csv under {d}")
        per = {}
        for fn in files:
            with open(fn) as f:
                for r in csv.DictReader(f):
                    if r["Counter_Name"] != counter:
                        continue
                    key = (r["Kernel_Name"], int(r["Dispatch_Id"]))
                    per[key] = per.get(key, 0.0) + float(r["Counter_Value"])
        return per

    def last_of(per, name):
        hits = [(did, v) for (k, did), v in per.items() if name in k]
        return max(hits)[1] if hits else None

    fetch, write = read(fetch_dir, "FETCH_SIZE"), read(write_dir, "WRITE_SIZE")
    probe_kib = probe_mib * 1024.0
    # the copy probe: the elementwise kernel that moved the most bytes
    fcopy = max(v for (k, _), v in fetch.items() if "elementwise" in k)
    wcopy = max(v for (k, _), v in write.items() if "elementwise" in k)
    fs, ws = probe_kib / fcopy, probe_kib / wcopy
    out = {}
    for k in TRAFFIC_KERNELS:
        fk, wk = last_of(fetch, k), last_of(write, k)
        if fk is not None and wk is not None:
            out[k] = (fk, wk, int(round((fk * fs + wk * ws) * 1024)))
    probe = {"mib": probe_mib, "fetch_kib": fcopy, "write_kib": wcopy, "fetch_scale": fs,
             "write_scale": ws}
    return out, probe


def record_traffic(fetch_dir: str, write_dir: str, probe_mib: int, commands):
    """Write profiles/traffic.json from two rocprofv3 --pmc runs of this bench
    (see traffic_from_counters); runs on the host from the counter files."""
    per, probe = traffic_from_counters(fetch_dir, write_dir, probe_mib)
    doc = {"_note": "HBM bytes per launch from rocprofv3 --pmc FETCH_SIZE and WRITE_SIZE runs "
                    "(KiB per dispatch, the last dispatch of each kernel), each scaled by the "
                    "reading of the same counter for an elementwise copy of "
                    f"{probe_mib} MiB read + {probe_mib} MiB written in the same run "
                    "(bench.py --copy-probe-mib); valid while the device sources hash to "
                    "device_sources_sha256",
           "copy_probe": probe}
    sha = device_sources_sha256()
    for k, (fk, wk, nbytes) in per.items():
        doc[k] = {"large:infra": {"device_sources_sha256": sha, "fetch_kib": fk, "write_kib": wk,
                                  "fetch_scale": probe["fetch_scale"],
                                  "write_scale": probe["write_scale"],
                                  "hbm_bytes_per_launch": nbytes, "commands": list(commands)}}
    path = os.path.join(ROOT, "profiles", "traffic.json")
    with open(path, "w") as f:
        json.dump(doc, f, indent=1)
        f.write("\n")
    return doc


def live_traffic(tune_path: str, log, timeout_s: float = 180.0):
    """HBM bytes per launch of the kernels measured in this run: the headline
    step once more in two child processes under rocprofv3 --pmc (FETCH_SIZE,
    then WRITE_SIZE), with this run's tuned choices (its tune cache) and a
    1 GiB copy probe for the scale.  Returns ({kernel: bytes}, the commands)
    or (None, reason) when rocprofv3 is missing or a run fails."""
    import shutil
    import subprocess
    import tempfile
    prof = shutil.which("rocprofv3") or ("/opt/rocm/bin/rocprofv3"
                                         if os.path.exists("/opt/rocm/bin/rocprofv3") else None)
    if prof is None:
        return None, "rocprofv3 not found"
    work = tempfile.mkdtemp(prefix="eis_pmc_", dir="/tmp")
    child = [sys.executable, os.path.abspath(__file__), "--steps", "1", "--warmup", "0",
             "--no-cpu-baseline", "--no-serving", "--no-configs", "--no-traffic",
             "--copy-probe-mib", "1024"]
    if tune_path:
        child += ["--tune-cache", tune_path]
    else:
        child += ["--no-tune"]
    dirs, cmds = [], []
    env = dict(os.environ, TMPDIR="/tmp")
    for counter in ("FETCH_SIZE", "WRITE_SIZE"):
        d = os.path.join(work, counter.lower())
        cmd = [prof, "--pmc", counter, "--output-format", "csv", "-d", d, "-o", "run", "--"] + child
        log(f"traffic: {counter} run")
        try:
            with open(os.path.join(work, counter.lower() + ".log"), "w") as lf:
                r = subprocess.run(cmd, cwd="/tmp", env=env, stdout=lf, stderr=subprocess.STDOUT,
                                   timeout=timeout_s)
        except subprocess.TimeoutExpired:
            return None, f"{counter} run timed out"
        # rocprofv3 itself may end with a fault after writing its results
        if r.returncode != 0 and not os.path.isdir(d):
            return None, f"{counter} run failed ({r.returncode})"
        dirs.append(d)
        cmds.append(" ".join(["rocprofv3", "--pmc", counter, "--", "python3", "bench.py"] +
                             child[2:]))
    try:
        per, _ = traffic_from_counters(dirs[0], dirs[1], 1024)
    except (RuntimeError, ValueError) as e:
        return None, f"counters unreadable: {e}"
    return {k: v[2] for k, v in per.items()}, cmds


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


def cpu_baseline_method(a: int, b: int, target_s: float = 8.0):
    """The method itself on the CPU (ref/: Algorithm Infrastructure with
    NUCOMP / NUDUPL, exact integers, all host threads) on a bounded random
    sample of the members of D in [a, b): the second CPU baseline, beside the
    oracle's plain definition."""
    import numpy as np
    import oracle
    import ref
    from paper_2507_06579_amd import workloads
    bits, _ = oracle.sqfree_range(a, b)
    n = oracle.num_candidates(a, b)
    d0 = oracle.first_candidate(a)
    idx = np.flatnonzero(np.unpackbits(bits, bitorder="little")[:n])
    members = (d0 + 8 * idx[workloads.sample_indices(idx.size, idx.size, seed=9)]).astype(np.int64)
    cores = os.cpu_count() or 1
    k0 = min(64 * cores, members.size)
    t = time.perf_counter()
    ref.classify_list(members[:k0], nthreads=cores)
    dt0 = max(time.perf_counter() - t, 1e-3)
    k = int(min(members.size - k0, max(cores, k0 * target_s / dt0)))
    sample = members[k0:k0 + k]
    t = time.perf_counter()
    flags, bad = ref.classify_list(sample, nthreads=cores)
    dt = time.perf_counter() - t
    return {"value": round(sample.size / dt, 2), "unit": "discriminants/s", "cores": cores,
            "kind": "method (CPU, Algorithm Infrastructure with NUCOMP/NUDUPL, int64/int128)",
            "sample": f"{sample.size} random members of D in [{a}, {b}) ({dt:.1f} s on {cores} "
                      f"threads of {cpu_model()}; {bad} failed a check; {int(flags.sum())} in E)"}


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

def stats_delta(st1, st0):
    """Counters of eis_get_stats accumulated between two snapshots."""
    out = {}
    for k, v in st1.items():
        if isinstance(v, list):
            out[k] = [x - y for x, y in zip(v, st0[k])]
        elif isinstance(v, (int, float)) and k in st0:
            out[k] = v - st0[k]
    return out


def slot_model(eis, name, d):
    """(VALU issue slots, units of work, unit name, model details) of the
    work a walk kernel did, from the counters `d` (a stats_delta)."""
    k = eis.KERNELS.index(name)
    ks, kl = d["kernel_steps"], max(1, d["kernel_launches"][k])
    if name == "walk_window":
        work = {"rho_steps": ks[k], "entries": d["window_entries"]}
        slots = sum(WINDOW_SLOTS[key] * v for key, v in work.items())
        return (slots, ks[k], "rho step",
                {"slots": WINDOW_SLOTS,
                 "work_per_launch": {key: int(v / kl) for key, v in work.items()}})
    if name != "walk_giant":
        return VALU_SLOTS_PER_STEP[name] * ks[k], ks[k], "rho step", None
    work = {key: d["giant_" + key]
            for key in ("compositions", "gcd_branches", "xgcd_steps", "reduce_steps",
                        "lookups")}
    work["partial_euclid_steps"] = d["giant_euclid_steps"] - d["giant_xgcd_steps"]
    work["walk_steps"] = ks[k]
    slots = sum(GIANT_SLOTS[key] * v for key, v in work.items())
    fill = {}
    for ph in ("compose", "walk"):
        nph, nln = d[f"giant_{ph}_phases"], d[f"giant_{ph}_lanes"]
        fill[ph] = {"phases_per_launch": int(nph / kl),
                    "busy_lanes_per_phase": round(nln / max(1, nph), 2)}
    return (slots, work["compositions"],
            "giant step (composition, reduction, walk to a distinguished ideal, lookup)",
            {"slots": GIANT_SLOTS,
             "work_per_launch": {key: int(v / kl) for key, v in work.items()},
             "phase_fill": fill})


WALKS = ["walk_plain", "walk_handoff", "walk_window", "walk_giant"]
KERNEL_NAME = {"walk_plain": "k_walk_baby", "walk_handoff": "k_walk_baby",
               "walk_window": "k_walk_window", "walk_giant": "k_walk_giant"}


def walk_rooflines(eis, d):
    """Per walk kernel with timed launches in `d`: achieved VALU lane-slots/s
    (model slots of its counted work / its summed event time) and the
    fraction of the peak; the dominant kernel (longest) first."""
    out = {}
    for name in WALKS:
        k = eis.KERNELS.index(name)
        ms, nl = d["kernel_ms"][k], d["kernel_launches"][k]
        if not nl or ms <= 0 or not d["kernel_steps"][k]:
            continue
        slots, units, uw, md = slot_model(eis, name, d)
        ach = slots / (ms / 1e3)
        ent = {"kernel": KERNEL_NAME[name], "bound": "alu", "achieved": round(ach / 1e12, 3),
               "peak": round(PEAK_LANE_OPS / 1e12, 3), "unit": "T VALU lane-slots/s",
               "frac": round(ach / PEAK_LANE_OPS, 4), "ms": round(ms, 3), "launches": nl,
               "ops_per_unit": round(slots / max(1, units), 1), "unit_of_work": uw,
               "units": int(units)}
        if md:
            ent["model"] = md
        out[name] = ent
    return dict(sorted(out.items(), key=lambda kv: -kv[1]["ms"]))


def oracle_rate(members, target_s: float):
    """The oracle on a prefix of `members` (a shuffled array of members of D)
    sized for about target_s seconds on all host cores: (discriminants/s,
    sample size, seconds, rho steps)."""
    import oracle
    cores = os.cpu_count() or 1
    k0 = min(4 * cores, members.size)
    t = time.perf_counter()
    oracle.classify_list(members[:k0], nthreads=cores)
    dt0 = max(time.perf_counter() - t, 1e-3)
    k = int(min(members.size - k0, max(cores, k0 * target_s / dt0)))
    if k <= 0:
        return k0 / dt0, k0, dt0, 0
    sample = members[k0:k0 + k]
    t = time.perf_counter()
    _, steps = oracle.classify_list(sample, nthreads=cores)
    dt = time.perf_counter() - t
    return sample.size / dt, int(sample.size), dt, int(steps)


def members_of(ranges, total: int, seed: int):
    """A shuffled array of about `total` members of D drawn from the given
    ranges, each range contributing in proportion to its number of
    candidates (uniformly within it); the oracle's sieve finds them."""
    import numpy as np
    import oracle
    rng = np.random.default_rng(seed)
    ncand = [oracle.num_candidates(a, b) for a, b in ranges]
    tot = max(1, sum(ncand))
    out = []
    for (a, b), n in zip(ranges, ncand):
        want = int(round(total * n / tot))
        if n == 0 or want == 0:
            continue
        # a window of candidates around 1.3 times the wanted count (about
        # 0.81 of the candidates are in D), placed at random in the range
        m = min(n, int(want * 1.3) + 64)
        start = int(rng.integers(0, n - m + 1))
        d0 = oracle.first_candidate(a) + 8 * start
        bits, _ = oracle.sqfree_range(d0, d0 + 8 * m)
        idx = np.flatnonzero(np.unpackbits(bits, bitorder="little")[:m])
        if idx.size > want:
            idx = rng.choice(idx, want, replace=False)
        out.append(d0 + 8 * idx.astype(np.uint64))
    arr = np.concatenate(out) if out else np.zeros(0, dtype=np.uint64)
    rng.shuffle(arr)
    return arr


def cpu_sample(members, target_s: float, what: str):
    rate, k, dt, steps = oracle_rate(members, target_s)
    cores = os.cpu_count() or 1
    return {"value": round(rate, 2), "unit": "discriminants/s", "cores": cores, "kind": "oracle",
            "sample": f"{k} random members of D from {what}, full-period walk ({steps} rho "
                      f"steps, {dt:.1f} s on {cores} threads of {cpu_model()})"}


def measure_configs(eis, tune_path, cpu: bool, log, serving: bool = True):
    """The other measurement configurations: time, discriminants/s and the
    walk kernels' roofline fractions of each, and the oracle's rate on a
    bounded sample of the same workload."""
    import numpy as np
    from paper_2507_06579_amd import serve, workloads
    out = {}
    kt = eis.EIS_FLAG_KERNEL_TIMES

    def timed_count(ctx, a, b, reps):
        ctx.eis_count(a, b)
        s0 = ctx.eis_get_stats()
        best = float("inf")
        for _ in range(reps):
            t = time.perf_counter()
            r = ctx.eis_count(a, b)
            best = min(best, time.perf_counter() - t)
        d = stats_delta(ctx.eis_get_stats(), s0)
        for key, v in d.items():  # per call
            d[key] = [x / reps for x in v] if isinstance(v, list) else v / reps
        return r, best, d

    # d1: the plain walk on [5, 10^6]
    a, b = workloads.SMALL
    log(f"config d1: [{a}, {b}) plain walk")
    with eis.Context(method=eis.Method.BABY, flags=kt) as c:
        (n_sq, n_e), dt, d = timed_count(c, a, b, 5)
    out["d1"] = {"workload": f"plain walk, all d = 5 mod 8 in [{a}, {b})", "pi_D": n_sq,
                 "pi_E": n_e, "ms": round(dt * 1e3, 3),
                 "discriminants_per_s": round(n_sq / dt, 1),
                 "roofline": walk_rooflines(eis, d)}
    if cpu:
        import oracle
        t = time.perf_counter()
        r = oracle.classify_range(a, b, want_bits=False)
        dtc = time.perf_counter() - t
        assert (r["n_sqfree"], r["n_eis"]) == (n_sq, n_e)
        out["d1"]["cpu_baseline"] = {
            "value": round(n_sq / dtc, 2), "unit": "discriminants/s",
            "cores": os.cpu_count() or 1, "kind": "oracle",
            "sample": f"the whole range ({r['steps']} rho steps, {dtc:.2f} s on "
                      f"{os.cpu_count() or 1} threads of {cpu_model()}); same counts"}

    # d2: plain walk against giant steps at 10^9
    a, b = workloads.MID
    out["d2"] = {"workload": f"all d = 5 mod 8 in [{a}, {b}), both methods"}
    bits = {}
    for label, method in (("baby", eis.Method.BABY), ("infra", eis.Method.INFRA)):
        log(f"config d2: [{a}, {b}) {label}")
        with eis.Context(method=method, flags=kt) as c:
            r = c.eis_classify(a, b)
            (n_sq, n_e), dt, d = timed_count(c, a, b, 5)
        bits[label] = (bytes(r[0]), bytes(r[1]), r[2], r[3])
        out["d2"][label] = {"ms": round(dt * 1e3, 3), "discriminants_per_s": round(n_sq / dt, 1),
                            "executed_rho_steps_per_s": round(d["baby_steps"] / dt, 1),
                            "roofline": walk_rooflines(eis, d)}
    if bits["baby"] != bits["infra"]:
        raise SystemExit("d2: the two methods' bitmaps differ")
    out["d2"]["pi_D"], out["d2"]["pi_E"] = bits["baby"][2], bits["baby"][3]
    out["d2"]["identical_bitmaps"] = True
    if cpu:
        out["d2"]["cpu_baseline"] = cpu_sample(members_of([(a, b)], 2000000, 11), 5.0,
                                               f"[{a}, {b})")

    # d3: 64 uneven ranges, one batched call against 64 single calls
    ranges = workloads.batch_ranges()
    ra, rb = [x for x, _ in ranges], [y for _, y in ranges]
    log("config d3: 64 uneven ranges, batched and one by one")
    with eis.Context(tune_cache_path=tune_path) as c:
        c.eis_count_batch(ra, rb)
        s0 = c.eis_get_stats()
        tb = float("inf")
        for _ in range(3):
            t = time.perf_counter()
            sb, eb = c.eis_count_batch(ra, rb)
            tb = min(tb, time.perf_counter() - t)
        t = time.perf_counter()
        singles = [c.eis_count(x, y) for x, y in ranges]
        ts = time.perf_counter() - t
    batched = [(int(x), int(y)) for x, y in zip(sb, eb)]
    if batched != singles:
        raise SystemExit("d3: batched and single counts differ")
    with eis.Context(tune_cache_path=tune_path, flags=kt | eis.EIS_FLAG_NO_GRAPHS) as c:
        c.eis_count_batch(ra, rb)
        s0 = c.eis_get_stats()
        c.eis_count_batch(ra, rb)
        dk = stats_delta(c.eis_get_stats(), s0)
    n_d = sum(x for x, _ in batched)
    out["d3"] = {"workload": f"64 ranges, start log-uniform in [1e6, 1e11], width log-uniform "
                             f"in [1e4, 1e7], seed {workloads.BATCH_SEED}",
                 "members_of_D": n_d, "pi_E": sum(y for _, y in batched),
                 "batched_ms": round(tb * 1e3, 3), "singles_ms": round(ts * 1e3, 3),
                 "batched_discriminants_per_s": round(n_d / tb, 1),
                 "singles_discriminants_per_s": round(n_d / ts, 1),
                 "identical_counts": True,
                 "roofline": walk_rooflines(eis, dk)}
    if cpu:
        out["d3"]["cpu_baseline"] = cpu_sample(members_of(ranges, 1500000, 13), 5.0,
                                               "the 64 ranges (in proportion to their widths)")

    if not serving:
        return out
    # d5: serving, open-loop Poisson arrivals swept past saturation
    sweep = []
    srv_members = None
    with eis.Context(serve_slots=256, tune_cache_path=tune_path) as c:
        for rate in (10.0, 100.0, 1000.0, 3000.0, 10000.0):
            n = int(min(2000, max(20, rate * 3.0)))
            reqs = workloads.serve_requests(n, rate)
            log(f"config d5: {n} requests at {rate:g} req/s")
            s0 = c.eis_get_stats()
            res = serve.run_open_loop(c, reqs)
            d = stats_delta(c.eis_get_stats(), s0)
            row = {"rate_req_s": rate}
            row.update(serve.summarize(res, reqs))
            # the walk work done over the run's wall time, against the peak
            slots = sum(slot_model(eis, name, d)[0] for name in WALKS)
            row["walk_frac_of_peak_over_wall_time"] = round(slots / res["wall_s"] / PEAK_LANE_OPS, 4)
            row["saturated"] = row["throughput_req_s"] < 0.9 * rate
            sweep.append(row)
            if srv_members is None or len(reqs) > len(srv_members):
                srv_members = [(x, y) for _, x, y in reqs]
    sat = [r["rate_req_s"] for r in sweep if r["saturated"]]
    out["d5"] = {"workload": "range counts [a, a+w), a log-uniform in [1e6, 1e11], w log-uniform "
                             f"in [1e3, 1e7], seed {workloads.SERVE_SEED}",
                 "sweep": sweep,
                 "max_throughput_req_s": max(r["throughput_req_s"] for r in sweep),
                 "first_saturated_rate_req_s": sat[0] if sat else None}
    if cpu:
        out["d5"]["cpu_baseline"] = cpu_sample(members_of(srv_members, 1500000, 17), 5.0,
                                               "the requested ranges (in proportion to their "
                                               "widths)")
    return out


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
    ap.add_argument("--tune-cache", default=None,
                    help="auto method with the choices of this tune cache (no tuning)")
    ap.add_argument("--no-traffic", action="store_true",
                    help="do not measure the dominant kernel's HBM traffic in child "
                         "rocprofv3 runs (then it comes from profiles/traffic.json, if current)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-serving", action="store_true",
                    help="skip the serving sweep (config d5)")
    ap.add_argument("--no-configs", action="store_true",
                    help="measure the headline workload only (no d1-d3, d5)")
    ap.add_argument("--record-traffic", nargs=2, metavar=("FETCH_DIR", "WRITE_DIR"),
                    help="write profiles/traffic.json from the output folders of two "
                         "rocprofv3 --pmc runs (FETCH_SIZE, WRITE_SIZE) of this bench with "
                         "--copy-probe-mib (given here too), then exit; no GPU is used")
    ap.add_argument("--traffic-command", action="append", default=[],
                    help="with --record-traffic: a command line to record beside the counts")
    args = ap.parse_args()
    if args.record_traffic:
        doc = record_traffic(args.record_traffic[0], args.record_traffic[1],
                             args.copy_probe_mib or 1024, args.traffic_command)
        for k in TRAFFIC_KERNELS:
            if k in doc:
                print(f"{k}: {doc[k]['large:infra']['hbm_bytes_per_launch'] / 1e9:.3f} GB per launch")
        return
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
    import tempfile
    if args.tune_cache:
        tune_path = args.tune_cache
    else:
        tune_dir = tempfile.mkdtemp(prefix="eis_tune_")
        tune_path = os.path.join(tune_dir, "tune.json")
    ctx = eis.Context(device=0, method=method, flags=eis.EIS_FLAG_KERNEL_TIMES,
                      window_scale=args.window_scale, tune_cache_path=tune_path)
    if method == eis.Method.AUTO and not args.no_tune and not args.tune_cache:
        t = time.perf_counter()
        ctx.eis_tune()
        log(f"autotuner: {time.perf_counter() - t:.1f} s")
    chosen, wscale = ctx.eis_tuned_choice(a)
    wchunk, pass_cand = ctx.eis_tuned_shape(a)
    log(f"method at d={a}: {chosen.name}, window scale {wscale}, walk chunk {wchunk}, "
        f"pass {pass_cand} candidates")
    if os.path.exists(tune_path):
        with open(tune_path) as f:
            tune_doc = json.load(f)
        for bn in tune_doc["bins"]:
            log(f"tuner bin {bn}")

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
                for key in ("compositions", "gcd_branches", "xgcd_steps", "reduce_steps",
                            "lookups")}
        work["partial_euclid_steps"] = (st["giant_euclid_steps"] - base["giant_euclid_steps"]
                                        - work["xgcd_steps"])
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
                   "window_scale": wscale, "walk_chunk": wchunk,
                   "pass_candidates": pass_cand},
        "baby_steps_per_s": round(baby / elapsed, 1),
        "fallbacks_per_step": (st["fallbacks"] - base["fallbacks"]) // args.steps,
        "giant_steps_per_s": round(giant / elapsed, 1),
        "kernels": kernels,
        "roofline": roofline,
        "roofline_other_walks": others,
    }
    ctx.close()
    roofline["traffic_source"] = None
    if roofline["traffic"] is not None:
        roofline["traffic_source"] = "profiles/traffic.json (recorded for these device sources)"
    if not args.no_traffic:
        per, how = live_traffic(tune_path if os.path.exists(tune_path) else None, log)
        if per is not None and roofline["kernel"] in per:
            roofline["traffic"] = per[roofline["kernel"]]
            roofline["traffic_source"] = "measured in this run: " + " ; ".join(how)
            for name, ent in others.items():
                kn = KERNEL_NAME.get(name)
                if kn in per:
                    ent["traffic"] = per[kn]
            log(f"traffic: {roofline['traffic'] / 1e9:.2f} GB per launch of {roofline['kernel']}")
        else:
            log(f"traffic not measured: {how}")
    if not args.no_configs:
        if not os.path.exists(tune_path):
            tune_path = None  # untuned: the contexts of the configs take the defaults
        cfgs = measure_configs(eis, tune_path, not args.no_cpu_baseline, log,
                               serving=not args.no_serving)
        out["configs"] = cfgs
        if "d5" in cfgs:
            row = next(r for r in cfgs["d5"]["sweep"] if r["rate_req_s"] == 100.0)
            out["p99_query_latency_ms"] = row["p99_ms"]
            out["serving"] = dict(row, workload=cfgs["d5"]["workload"])
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle on a bounded sample)")
        out["cpu_baseline"] = cpu_baseline(a, b)
        log("cpu baseline of the method (ref/ on a bounded sample)")
        out["cpu_baseline_method"] = cpu_baseline_method(a, b)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
