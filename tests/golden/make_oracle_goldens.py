"""Write the oracle's results for the full-size windows to oracle_windows.json.

Every value in the output comes from ``oracle/`` (the plain full-period
continued-fraction walk and the range sieve over p^2) on the ranges of
``paper_2507_06579_amd.workloads``, which hold no arithmetic of the method.
Nothing here loads or calls the HIP library.

Entries:
  windows   the plain-vs-infrastructure window [10^9, 10^9 + 10^7), the
            Table 1 window [10^11 - 10^8, 10^11) and the window
            [10^12 - 2^26, 10^12) at the top of the supported heights: pi_D,
            pi_E and the sha256 of the packed squarefree and Eisenstein
            bitmaps (bit i of byte i/8, LSB first, is the candidate
            d0 + 8i, d0 the least d >= a with d = 5 mod 8);
  batch     (a, b, pi_D, pi_E) of each of the 64 seeded uneven ranges;
  serve     (a, b, pi_D, pi_E) of the first 48 requests of the seeded
            serving stream.

Usage:  python tests/golden/make_oracle_goldens.py [--only NAME ...] [--threads N]
The file is updated entry by entry, so an interrupted run keeps what it
finished.  The full set takes about an hour of one 8-core host.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_2507_06579_amd import workloads  # noqa: E402

OUT = os.path.join(HERE, "oracle_windows.json")

WINDOWS = {
    "mid_1e9": workloads.MID,
    "table1_1e11": workloads.LARGE,
    "top_1e12": (10**12 - 2**26, 10**12),
}
N_SERVE = 48
SERVE_RATE = 100.0


def _load():
    if os.path.exists(OUT):
        with open(OUT) as f:
            return json.load(f)
    return {"windows": {}, "batch": None, "serve": None}


def _save(doc):
    tmp = OUT + ".tmp"
    with open(tmp, "w") as f:
        json.dump(doc, f, indent=1, sort_keys=True)
        f.write("\n")
    os.replace(tmp, OUT)


def _window(a, b, threads):
    n = oracle.num_candidates(a, b)
    nb = (n + 7) // 8
    r = oracle.classify_range(a, b, nthreads=threads)
    sq = bytes(r["sq_bits"][:nb])
    eb = bytes(r["eis_bits"][:nb])
    return {
        "a": a, "b": b, "n_cand": n,
        "n_sqfree": r["n_sqfree"], "n_eis": r["n_eis"],
        "sha256_sqfree": hashlib.sha256(sq).hexdigest(),
        "sha256_eis": hashlib.sha256(eb).hexdigest(),
        "oracle_steps": r["steps"],
    }


def _ranges(rs, threads):
    out = []
    for a, b in rs:
        r = oracle.classify_range(a, b, nthreads=threads, want_bits=False)
        out.append([a, b, r["n_sqfree"], r["n_eis"]])
    return out


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--only", nargs="*", default=None,
                    help="subset of: " + " ".join(list(WINDOWS) + ["batch", "serve"]))
    ap.add_argument("--threads", type=int, default=os.cpu_count() or 1)
    args = ap.parse_args(argv)
    names = args.only or (list(WINDOWS) + ["batch", "serve"])
    oracle.build(force=False)
    doc = _load()
    for name in names:
        t0 = time.time()
        if name in WINDOWS:
            doc["windows"][name] = _window(*WINDOWS[name], args.threads)
        elif name == "batch":
            doc["batch"] = {"seed": workloads.BATCH_SEED,
                            "ranges": _ranges(workloads.batch_ranges(), args.threads)}
        elif name == "serve":
            reqs = workloads.serve_requests(N_SERVE, SERVE_RATE)
            doc["serve"] = {"seed": workloads.SERVE_SEED, "rate": SERVE_RATE,
                            "ranges": _ranges([(a, b) for _, a, b in reqs], args.threads)}
        else:
            raise SystemExit(f"unknown entry {name}")
        _save(doc)
        print(f"{name}: {time.time() - t0:.1f} s", flush=True)


if __name__ == "__main__":
    main()
