"""GPU tests of the autotuner (method and window-scale choice per height).

The tuner changes only timing: every choice must give the same bits, which
the plain walk (itself pinned to the oracle by the parity tests) fixes.
"""
import json
import sys

import pytest

import paper_2507_06579_amd as eis

pytestmark = pytest.mark.gpu

SCALES = {1.0, 1.5, 1.75, 2.0, 2.25, 2.5, 3.5, 5.0}


def _say(msg):
    print(f"[gpu-tune] {msg}", flush=True)
    sys.stdout.flush()


def test_tune_choices_cache_and_bits(tmp_path):
    path = str(tmp_path / "tune.json")
    heights = [10**5, 3 * 10**6, 10**8, 4 * 10**9, 10**11, 10**12 - 10**6]
    with eis.Context(tune_cache_path=path) as c:
        _say("tuning")
        c.eis_tune()
        choices = [c.eis_tuned_choice(d) for d in heights]
        for m, w in choices:
            assert m in (eis.Method.BABY, eis.Method.INFRA)
            assert w in SCALES
        assert choices[0][0] == eis.Method.BABY  # below 10^6
        # the bits do not depend on the choice
        ranges = [(10**8, 10**8 + 10**6), (10**11 - 4 * 10**6, 10**11), (10**12 - 10**6, 10**12)]
        tuned = [c.eis_classify(a, b) for a, b in ranges]
    with open(path) as f:
        doc = json.load(f)
    assert doc["arch"] == "gfx950" and len(doc["bins"]) == 25
    assert set(doc["scales"]) == SCALES
    for bn in doc["bins"]:
        assert bn["walk_chunk"] in (8, 16, 32) and bn["pass_log2"] in (22, 23, 24)
        if bn["b"] >= 12 and bn["b"] < 24:
            # every timing behind the choice is recorded, and the scale kept
            # is the fastest one timed
            assert min(bn["pass_ms_24_23_22"]) > 0
            assert len(bn["scale_ms"]) == len(SCALES) and min(bn["scale_ms"]) > 0
            # (the cache prints times to 0.001 ms, so two scales can tie
            # there; the one kept must be one of the fastest)
            kept = bn["scale_ms"][doc["scales"].index(bn["window_scale"])]
            assert kept == pytest.approx(min(bn["scale_ms"]), abs=1e-3)
            assert bn["giant_ms"] == pytest.approx(min(bn["scale_ms"]), abs=1e-3)
            if bn["method"] == 1:
                assert min(bn["chunk_ms_8_16_32"]) > 0
    with eis.Context(method=eis.Method.BABY) as c:
        plain = [c.eis_classify(a, b) for a, b in ranges]
    for (sq1, e1, n1, m1), (sq2, e2, n2, m2) in zip(tuned, plain):
        assert (n1, m1) == (n2, m2)
        assert bytes(sq1) == bytes(sq2) and bytes(e1) == bytes(e2)
    # a new context loads the cache, shapes included
    with eis.Context(tune_cache_path=path) as c:
        assert [c.eis_tuned_choice(d) for d in heights] == choices
        shapes = [c.eis_tuned_shape(d) for d in heights]
    byb = {x["b"]: x for x in doc["bins"]}
    for d, (ch, ps) in zip(heights, shapes):
        b = max(k for k, x in byb.items() if x["from"] <= d)
        assert (ch, ps) == (byb[b]["walk_chunk"], 2 ** byb[b]["pass_log2"]), d
    # an explicit method and scale win over the tuned choice
    with eis.Context(tune_cache_path=path, method=eis.Method.INFRA, window_scale=2.75) as c:
        assert c.eis_tuned_choice(10**11) == (eis.Method.INFRA, 2.75)


def test_untuned_defaults():
    with eis.Context() as c:
        assert c.eis_tuned_choice(10**6)[0] == eis.Method.BABY
        assert c.eis_tuned_choice(10**11)[0] == eis.Method.INFRA
        assert c.eis_tuned_choice(10**11)[1] == 2.0


def test_tune_cache_rejects_partial_file(tmp_path):
    path = tmp_path / "bad.json"
    path.write_text('{"arch": "gfx950", "bins": [{"b": 12, "method": 1, "window_scale": 2.5}]}')
    with eis.Context(tune_cache_path=str(path)) as c:
        # not every bin present: defaults stay in force
        assert c.eis_tuned_choice(10**6) == (eis.Method.BABY, 2.0)


def test_kernel_times_and_step_counts():
    a, b = 10**11 - 4 * 10**6, 10**11
    for method in (eis.Method.BABY, eis.Method.INFRA):
        with eis.Context(method=method, flags=eis.EIS_FLAG_KERNEL_TIMES) as c:
            c.eis_count(a, b)
            st = c.eis_get_stats()
        ks, kl, kms = st["kernel_steps"], st["kernel_launches"], st["kernel_ms"]
        assert sum(ks) == st["baby_steps"] > 0
        k = eis.KERNELS
        assert kl[k.index("sieve")] == 1 and kl[k.index("popcount")] == 1
        gw = [st[f] for f in ("giant_compositions", "giant_euclid_steps", "giant_reduce_steps",
                              "giant_gcd_branches", "giant_lookups", "giant_xgcd_steps")]
        if method == eis.Method.BABY:
            assert kl[k.index("walk_plain")] == 1 and kl[k.index("walk_window")] == 0
            assert ks[k.index("walk_plain")] == st["baby_steps"]
            assert gw == [0, 0, 0, 0, 0, 0] and st["window_entries"] == 0
        else:
            assert kl[k.index("walk_window")] >= 1 and kl[k.index("walk_giant")] >= 1
            assert kl[k.index("giant_square")] == kl[k.index("walk_giant")]
            assert ks[k.index("walk_window")] > 0 and st["giant_steps"] > 0
            comps, euclid, red, gcdb, looks, xgcd = gw
            # every giant ideal (g, g2 and each composition) is looked up
            # once, unless a check fails first; every composition runs at
            # least one Euclid step, and some take NUCOMP's gcd branch; the
            # extended Euclid's steps are part of the Euclid steps
            assert 0 < comps < st["giant_steps"] and 0 < looks <= st["giant_steps"]
            assert looks >= comps and euclid > comps and 0 <= gcdb < comps and red >= 0
            assert comps < xgcd < euclid
            # the window walk appends its distinguished ideals (Q = 2 mod 64):
            # about one reduction step in 16
            ent = st["window_entries"]
            assert 0.04 < ent / ks[k.index("walk_window")] < 0.09
            # the giant walk runs its d's in phases of at most 64 busy lanes:
            # every lookup belongs to a compose phase, every walk step to a
            # walk phase
            for ph in ("compose", "walk"):
                nph, nln = st[f"giant_{ph}_phases"], st[f"giant_{ph}_lanes"]
                assert 0 < nph and nph <= nln <= 64 * nph
            assert st["giant_compose_lanes"] >= looks
            assert st["giant_walk_lanes"] * 16 >= ks[k.index("walk_giant")]
        assert all(x >= 0 for x in kms)
        assert 0 < sum(kms) <= st["last_total_ms"] * 1.05 + 0.5
    # without the flag nothing is timed
    with eis.Context() as c:
        c.eis_count(10**9, 10**9 + 10**5)
        assert sum(c.eis_get_stats()["kernel_launches"]) == 0
