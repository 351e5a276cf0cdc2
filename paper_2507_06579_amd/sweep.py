"""Paper-scale sweep: pi_D(x) and pi_E(x) for x up to 10^11 (Section 3.1), and
the same counts over the prime subsequence (Section 3.2, prime subsequence).

The range [0, X) is cut into segments whose ends include every power of ten;
segments go to the GPU through eis_count_batch a few at a time, and after
every batch the finished segments are written to a JSON checkpoint, so that
an interrupted sweep resumes where it stopped.  From the segment counts the
sweep reports

  * pi_D(10^k) and pi_E(10^k) for every power of ten up to X;
  * the coefficient c of the fitted law pi_E(x) ~ x / (3 pi^2) + c x^(5/6)
    (the paper reports c = -0.024 from its own sweep to 10^11), by least
    squares over the cumulative counts at every segment end above 10^6;
  * per segment, the share P(d in E | d in D) next to the paper's
    1/3 - 0.201 / d^(1/6), averaged over the segment.

With --primes the set is D restricted to primes (primes p = 5 mod 8), and the
sweep reports pi_{D cap P}(10^k), pi_{E cap P}(10^k) and the coefficient c of
    pi_{E cap P}(x) ~ pi(x) / 12 + c * Li6(x),  Li6(x) = int_2^x dt / (t^(1/6) log t)
(the paper quotes c = -0.037 from the sweep it cites), with pi(x)/4 taken as
the measured pi_{D cap P}(x): the two differ by the Chebyshev bias between
residue classes mod 8, far below the x^(5/6)/log x term.  Per segment, the
share P(p in E | p in D cap P) stands next to 1/3 - 0.148 / p^(1/6), the law
weighted by the prime density 1/log t over the segment.

All counting runs in libeis.so; this module only plans, checkpoints and
summarises.

  python -m paper_2507_06579_amd.sweep --max 1e11 --checkpoint sweep.json
  python -m paper_2507_06579_amd.sweep --max 1e11 --primes --checkpoint primes.json
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

PAPER_C56 = -0.024       # Section 3.1, the fitted coefficient of x^(5/6)
PAPER_DENSITY_B = 0.201  # Section 3.1, P(E | D) ~ 1/3 - b / d^(1/6)
PAPER_PRIME_C = -0.037   # Section 3.2, prime subsequence: coefficient of Li6(x)
PAPER_PRIME_B = 0.148    # Section 3.2, prime subsequence: P(E | D cap P) ~ 1/3 - b / p^(1/6)

SETS = ("squarefree", "prime")


def segments(xmax: int, width: int):
    """Half-open segments [a, b) covering [0, xmax): powers of ten up to
    `width` are segment ends, then steps of `width` (also hitting every
    power of ten above it)."""
    ends = []
    p = 10
    while p < min(width, xmax):
        ends.append(p)
        p *= 10
    x = width
    while x < xmax:
        ends.append(x)
        x += width
    ends.append(xmax)
    out, a = [], 0
    for b in sorted(set(ends)):
        if b > a:
            out.append((a, b))
            a = b
    return out


def load_checkpoint(path: str, xmax: int, width: int, which: str = "squarefree"):
    if not path or not os.path.exists(path):
        return {}
    with open(path) as f:
        doc = json.load(f)
    if (doc.get("max") != xmax or doc.get("width") != width
            or doc.get("set", "squarefree") != which):
        raise SystemExit(f"{path} belongs to another sweep (max {doc.get('max')}, "
                         f"width {doc.get('width')}, set {doc.get('set', 'squarefree')})")
    return {(int(s["a"]), int(s["b"])): (int(s.get("n_set", s.get("n_sqfree"))), int(s["n_eis"]))
            for s in doc["segments"]}


def save_checkpoint(path: str, xmax: int, width: int, done: dict, which: str = "squarefree"):
    if not path:
        return
    doc = {"max": xmax, "width": width, "set": which,
           "segments": [{"a": a, "b": b, "n_set": s, "n_eis": e}
                        for (a, b), (s, e) in sorted(done.items())]}
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(doc, f)
    os.replace(tmp, path)


def mean_inv_sixth_root(a: int, b: int) -> float:
    """Mean of d^(-1/6) over [max(a, 5), b) (for the density law)."""
    lo = max(a, 5)
    if b <= lo:
        return 0.0
    return (1.2 * (b ** (5 / 6) - lo ** (5 / 6))) / (b - lo)


def expint_ei(z: float) -> float:
    """Ei(z) for z > 0 by its power series gamma + log z + sum z^k / (k k!);
    every term is positive, so the sum is accurate for the z <= 30 used here."""
    total, term, k = 0.0, 1.0, 0
    while True:
        k += 1
        term *= z / k
        add = term / k
        total += add
        if add < 1e-17 * total:
            break
    return 0.5772156649015329 + math.log(z) + total


def li6(x: float, lo: float = 2.0) -> float:
    """int_lo^x dt / (t^(1/6) log t) = Ei(5/6 log x) - Ei(5/6 log lo) (t = e^u)."""
    if x <= lo:
        return 0.0
    return expint_ei(5 / 6 * math.log(x)) - expint_ei(5 / 6 * math.log(lo))


def li(x: float, lo: float = 2.0) -> float:
    """int_lo^x dt / log t = Ei(log x) - Ei(log lo)."""
    if x <= lo:
        return 0.0
    return expint_ei(math.log(x)) - expint_ei(math.log(lo))


def prime_mean_inv_sixth_root(a: int, b: int) -> float:
    """Mean of p^(-1/6) over [max(a, 5), b) under the prime density 1/log t."""
    lo = max(a, 5)
    if b <= lo:
        return 0.0
    return li6(b, lo) / li(b, lo)


def fit_prime_c(points):
    """Least-squares c in pi_{E cap P}(x) - pi_{D cap P}(x)/3 = c Li6(x) over
    (x, pi_{D cap P}, pi_{E cap P})."""
    num = den = 0.0
    for x, pd, pe in points:
        t = li6(x)
        num += (pe - pd / 3) * t
        den += t * t
    return num / den if den else float("nan")


def fit_c56(points):
    """Least-squares c in pi_E(x) - x/(3 pi^2) = c x^(5/6) over (x, pi_E)."""
    num = den = 0.0
    for x, pe in points:
        t = x ** (5 / 6)
        num += (pe - x / (3 * math.pi ** 2)) * t
        den += t * t
    return num / den if den else float("nan")


def summarise(done: dict, xmax: int, which: str = "squarefree"):
    segs = sorted(done.items())
    cum_s = cum_e = 0
    powers, cumulative, density = [], [], []
    prime = which == "prime"
    for (a, b), (s, e) in segs:
        cum_s += s
        cum_e += e
        cumulative.append((b, cum_s, cum_e))
        if b == 10 ** round(math.log10(b)):
            if prime:
                powers.append({"x": b, "pi_DP": cum_s, "pi_EP": cum_e,
                               "c_at_x": round((cum_e - cum_s / 3) / li6(b), 5) if b > 2 else None})
            else:
                powers.append({"x": b, "pi_D": cum_s, "pi_E": cum_e,
                               "pi_D_over_x_pi2": round(cum_s * math.pi ** 2 / b, 6),
                               "c56_at_x": round((cum_e - b / (3 * math.pi ** 2)) / b ** (5 / 6), 5)})
        if s:
            law = (1 / 3 - PAPER_PRIME_B * prime_mean_inv_sixth_root(a, b) if prime
                   else 1 / 3 - PAPER_DENSITY_B * mean_inv_sixth_root(a, b))
            density.append({"a": a, "b": b, "share": round(e / s, 6), "paper_law": round(law, 6)})
    if prime:
        fit_pts = [(x, pd, pe) for x, pd, pe in cumulative if x >= 10 ** 6]
        c = fit_prime_c(fit_pts)
        return {"max": xmax, "set": which, "pi_DP": cum_s, "pi_EP": cum_e,
                "powers_of_ten": powers, "c_fit": round(c, 5), "c_paper": PAPER_PRIME_C,
                "b_fit": round(-4 * c, 5), "b_paper": PAPER_PRIME_B, "density": density}
    fit_pts = [(x, pe) for x, _, pe in cumulative if x >= 10 ** 6]
    return {"max": xmax, "set": which, "pi_D": cum_s, "pi_E": cum_e, "powers_of_ten": powers,
            "c56_fit": round(fit_c56(fit_pts), 5), "c56_paper": PAPER_C56,
            "density": density}


def run(xmax: int, width: int, checkpoint: str, per_call: int = 8, ctx=None, log=print,
        which: str = "squarefree", tune: bool = False):
    from . import _lib as eis
    if which not in SETS:
        raise ValueError(f"set must be one of {SETS}")
    code = eis.EIS_SET_PRIME if which == "prime" else eis.EIS_SET_SQUAREFREE
    done = load_checkpoint(checkpoint, xmax, width, which)
    todo = [sg for sg in segments(xmax, width) if sg not in done]
    log(f"[sweep] {len(done)} segments done, {len(todo)} to go")
    own = ctx is None
    if own:
        ctx = eis.Context()
    t0 = time.perf_counter()
    if tune:
        # method and window scale per half-decade of height (timed below)
        ctx.eis_tune()
        log(f"[sweep] autotuner: {time.perf_counter() - t0:.1f} s")
    st0 = ctx.eis_get_stats()
    try:
        for i in range(0, len(todo), per_call):
            part = todo[i:i + per_call]
            s, e = ctx.eis_count_batch_set(code, [a for a, _ in part], [b for _, b in part])
            for sg, x, y in zip(part, s, e):
                done[sg] = (int(x), int(y))
            save_checkpoint(checkpoint, xmax, width, done, which)
            log(f"[sweep] up to {part[-1][1]:.3e}: {len(done)} segments, "
                f"{time.perf_counter() - t0:.1f} s")
        st1 = ctx.eis_get_stats()
    finally:
        if own:
            ctx.close()
    out = summarise(done, xmax, which)
    out["seconds"] = round(time.perf_counter() - t0, 2)
    # work of this run (segments restored from a checkpoint are not in it):
    # members of D classified, reduction steps, giant steps, and the d's the
    # giant-step method handed to the plain walk
    out["work"] = {k: st1[k] - st0[k] for k in ("discriminants", "baby_steps", "giant_steps",
                                                 "fallbacks")}
    return out


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--max", type=float, default=1e11)
    ap.add_argument("--width", type=float, default=1e9, help="segment width above 10^9")
    ap.add_argument("--checkpoint", default="", help="JSON checkpoint (resume)")
    ap.add_argument("--out", default="", help="write the summary here (JSON)")
    ap.add_argument("--per-call", type=int, default=8, help="segments per eis_count_batch")
    ap.add_argument("--primes", action="store_true", help="sweep the prime subsequence")
    ap.add_argument("--tune", action="store_true",
                    help="run the autotuner first (about 1.5 s; the untuned defaults are as fast "
                         "on this sweep)")
    args = ap.parse_args(argv)
    xmax, width = int(args.max), int(args.width)
    res = run(xmax, width, args.checkpoint, args.per_call,
              log=lambda m: print(m, file=sys.stderr, flush=True),
              which="prime" if args.primes else "squarefree", tune=args.tune)
    text = json.dumps(res)
    if args.out:
        with open(args.out, "w") as f:
            f.write(text + "\n")
    brief = {k: v for k, v in res.items() if k != "density"}
    print(json.dumps(brief), flush=True)


if __name__ == "__main__":
    main()
