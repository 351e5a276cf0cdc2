"""CPU pins of the method itself (ref/: Algorithm Infrastructure with NUCOMP,
NUDUPL and NUCOMPchoose, in exact integers, written from Appendix A).

The oracle pins the flags by the plain definition; these tests pin the
method's arithmetic, against facts that do not come from the method:
  * its cycle of reduced ideals has the oracle's period, and its regulator
    equals ln of the oracle's big-integer fundamental unit;
  * every composition (ideal product, NUDUPL, NUCOMP), followed by reduction,
    returns a reduced ideal ON that cycle, whose distance and residue are the
    inputs' plus what the algorithm claims for gamma and the reduction steps
    (distance identity to rounding, residue identity exactly, modulo one
    regulator), with gamma a unit at 2 (Appendix A, the localisation
    argument after Theorem A.1);
  * the unit Algorithm Infrastructure returns lies at exactly one regulator
    (not eps^2 or eps^3, which would keep or break the flag by accident),
    and its flag equals the oracle's on all of D below 3*10^4 and on samples
    from 10^6 to 10^12;
  * planted mistakes (gamma's residue dropped, ln|gamma| dropped, a wrong
    half-period formula) are caught.
"""
import math

import numpy as np
import pytest

import oracle
import ref

# heights of the composition tests: small d's (short cycles, many small
# norms) up to 10^11; the reference period there is about 10^5 ideals
COMPOSE_DS = [1901, 7053, 10005, 123461, 1000005, 1000037, 100000005, 1000000005,
              10000000029, 99999999997]


def _member(d):
    """The least member of D at or above d."""
    d = oracle.first_candidate(d)
    while not oracle.in_D_trial(d):
        d += 8
    return d


def _ln_eps(d):
    """ln eps_d from the oracle's big-integer unit (x0 + y0 sqrt d)/2, or None
    when its digits are not returned."""
    _, x0, y0, _, _ = oracle.unit_bigint(d)
    if x0 is None:
        return None
    if x0 < 10**300:
        return math.log((x0 + y0 * math.sqrt(d)) / 2)
    # x0 = eps + eps' with |eps'| = 1/eps: ln eps = ln x0 to double precision
    return math.log(x0)


def test_cycle_period_and_regulator_against_the_oracle():
    rng = np.random.default_rng(5)
    ds = [d for d in range(5, 6000, 8) if oracle.in_D_trial(d)]
    ds += [_member(int(x) * 8 + 5) for x in rng.integers(10**5 // 8, 10**8 // 8, size=30)]
    for d in ds:
        cy = ref.cycle(d)
        _, period, _ = oracle.walk_mod2(d)
        assert cy["period"] == period, d
        le = _ln_eps(d)
        if le is not None:
            assert abs(cy["R"] - le) <= 1e-9 * max(1.0, le), (d, cy["R"], le)


def _compose_cases(cy, rng, n):
    m = cy["period"]
    pairs = [(int(rng.integers(0, m)), int(rng.integers(0, m))) for _ in range(n)]
    pairs += [(i, i) for i in map(int, rng.integers(0, m, size=n // 4))]
    small = [k for k in range(m) if cy["Q"][k] <= 50]
    if small:
        pairs += [(int(rng.choice(small)), int(rng.integers(0, m))) for _ in range(n // 4)]
    return pairs


def _check_compositions(d, n, rng, mode=0):
    """Compose random pairs of cycle ideals; return (paths seen, list of
    failures)."""
    cy = ref.cycle(d)
    R = cy["R"]
    _, _, S = oracle.walk_mod2(d)  # log eps (the oracle's Z/3 log-sum)
    where = {(int(q), int(p)): k for k, (q, p) in enumerate(zip(cy["Q"], cy["P"]))}
    paths, bad = {}, []
    for i, j in _compose_cases(cy, rng, n):
        r = ref.compose(d, int(cy["Q"][i]), int(cy["P"][i]), int(cy["Q"][j]), int(cy["P"][j]),
                        mode)
        paths[r["path"]] = paths.get(r["path"], 0) + 1
        if r["err"]:
            bad.append((d, i, j, "check", r))
            continue
        k = where.get((r["Q"], r["P"]))
        if k is None:
            bad.append((d, i, j, "not on the cycle", r))
            continue
        x = (cy["dist"][i] + cy["dist"][j] + r["shift"] - cy["dist"][k]) / R
        mult = round(x)
        if abs(x - mult) > 1e-6:
            bad.append((d, i, j, "distance", x))
            continue
        if (int(cy["res"][i]) + int(cy["res"][j]) + r["res"] - int(cy["res"][k]) - mult * S) % 3:
            bad.append((d, i, j, "residue", mult))
    return paths, bad


def test_every_composition_lands_on_the_cycle_at_its_distance_and_residue():
    rng = np.random.default_rng(11)
    seen = {}
    for d in COMPOSE_DS:
        paths, bad = _check_compositions(_member(d), 1000, rng)
        assert not bad, bad[:3]
        for p, c in paths.items():
            seen[p] = seen.get(p, 0) + c
    # every branch of NUCOMPchoose was exercised
    assert set(seen) == {"product", "nudupl", "nucomp"}
    assert min(seen.values()) >= 1500


def test_compositions_near_the_largest_height():
    # 10^12: the cycle has ~3*10^5 ideals; products run to about 2^50
    rng = np.random.default_rng(12)
    paths, bad = _check_compositions(_member(10**12 - 2**20), 1000, rng)
    assert not bad, bad[:3]
    assert paths.get("nucomp", 0) > 900


def test_nucomp_for_every_pair_lands_on_the_cycle_too():
    """The composition the GPU kernels use: NUCOMP for every pair, squares
    included (NUCOMP handles equal inputs through its gcd step), and NUCOMP
    without its partial reduction (an unbounded L) when a norm is <= 50,
    which is then the plain ideal product with gamma = the gcd of the norms
    and s.  It too returns cycle ideals at the claimed distance and residue,
    and for squares of large-norm ideals it returns NUDUPL's ideal."""
    rng = np.random.default_rng(13)
    for d in COMPOSE_DS + [10**12 - 2**20]:
        d = _member(d)
        paths, bad = _check_compositions(d, 400, rng, mode=1)
        assert not bad, bad[:3]
        assert set(paths) == {"nucomp"}
        cy = ref.cycle(d)
        for k in map(int, rng.integers(0, cy["period"], size=100)):
            q, p = int(cy["Q"][k]), int(cy["P"][k])
            a, b = ref.compose(d, q, p, q, p, 0), ref.compose(d, q, p, q, p, 1)
            assert a["err"] == b["err"] == 0
            assert (a["Q"], a["P"]) == (b["Q"], b["P"]), (d, q, p)
            if q > 50:
                assert a["path"] == "nudupl"
                assert abs(a["shift"] - b["shift"]) <= 1e-9 * cy["R"] and a["res"] == b["res"]


def _classify_against_oracle(ds):
    for d in ds:
        r = ref.classify(d)
        assert r["err"] == 0, (d, r)
        f, _, _ = oracle.walk_mod2(d)
        assert r["flag"] == f, d
        cy = ref.cycle(d)
        # the unit found is eps itself: exactly one regulator
        assert abs(r["eps_dist"] - cy["R"]) <= 1e-9 * cy["R"], (d, r["eps_dist"], cy["R"])


def test_method_flags_and_unit_on_all_small_D():
    ds = [d for d in range(5, 30000, 8) if oracle.in_D_trial(d)]
    assert len(ds) == 3040
    _classify_against_oracle(ds)


@pytest.mark.parametrize("h", [10**6, 10**8, 10**9, 10**10])
def test_method_flags_and_unit_at_height(h):
    rng = np.random.default_rng(h % 9973)
    ds = sorted({_member(int(x) * 8 + 5) for x in rng.integers(h // 8, (h + 10**7) // 8, 500)})
    _classify_against_oracle(ds)
    ends = {ref.classify(d)["end"] for d in ds}
    assert "hit" in ends  # the giant steps decided some of them


def test_method_flags_near_1e11_and_1e12():
    rng = np.random.default_rng(77)
    for h, k in ((10**11 - 10**8, 300), (10**12 - 2**26, 150)):
        ds = sorted({_member(int(x) * 8 + 5) for x in rng.integers(h // 8, (h + 10**7) // 8, k)})
        flags, bad = ref.classify_list(ds)
        assert bad == 0
        ref_flags = [oracle.walk_mod2(d)[0] for d in ds]
        assert list(map(bool, flags)) == ref_flags
        # at these heights almost every d is decided by giant steps
        runs = [ref.classify(d) for d in ds[:40]]
        assert sum(r["end"] == "hit" for r in runs) >= 35
        assert sum(r["giants"] for r in runs) > 40 * 10


def test_planted_mistakes_are_caught():
    rng = np.random.default_rng(21)
    d = _member(1000000005)
    # gamma's residue dropped: some composition's residue identity fails
    with ref.mutation(1):
        _, bad = _check_compositions(d, 200, rng)
    assert any(b[3] == "residue" for b in bad)
    # ln|gamma| dropped: the distance identity fails
    with ref.mutation(2):
        _, bad = _check_compositions(d, 200, rng)
    assert any(b[3] == "distance" for b in bad)
    # a wrong half-period formula: some flag differs from the oracle's
    ds = [x for x in range(5, 30000, 8) if oracle.in_D_trial(x)]
    with ref.mutation(3):
        wrong = sum(ref.classify(x)["flag"] != oracle.walk_mod2(x)[0] for x in ds)
    assert wrong > 0
    # and without a mutation everything holds again
    _, bad = _check_compositions(d, 100, rng)
    assert not bad
