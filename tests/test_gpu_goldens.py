"""GPU parity at full size: every configuration against the oracle's goldens.

``tests/golden/oracle_windows.json`` holds what the oracle (the plain
full-period walk, nothing of the HIP path) computed for the full windows --
pi_D, pi_E and the sha256 of both packed bitmaps -- and the counts of every
range of the 64-range batch and of the first 48 serving requests; the script
beside it wrote them.  Here the HIP path, through the C ABI, must reproduce
them exactly with every method, window scale, tuned choice, batch form and
graph setting.  Flags and counts are integers: tolerance 0.
"""
import hashlib
import json
import os
import sys
import time

import numpy as np
import pytest

import oracle
import paper_2507_06579_amd as eis
from paper_2507_06579_amd import workloads

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "oracle_windows.json")
with open(GOLDEN) as _f:
    G = json.load(_f)


def _say(msg):
    print(f"[gpu-golden] {msg}", flush=True)
    sys.stdout.flush()


def _check_window(name, sq, eb, ns, ne):
    w = G["windows"][name]
    nb = (w["n_cand"] + 7) // 8
    assert (ns, ne) == (w["n_sqfree"], w["n_eis"]), name
    assert hashlib.sha256(bytes(sq[:nb])).hexdigest() == w["sha256_sqfree"], name
    assert hashlib.sha256(bytes(eb[:nb])).hexdigest() == w["sha256_eis"], name


WINDOW_CASES = [
    (name, method, ws)
    for name in ("mid_1e9", "table1_1e11", "top_1e12")
    for method, ws in ((eis.Method.BABY, 0.0), (eis.Method.INFRA, 0.0),
                       (eis.Method.AUTO, 0.0), (eis.Method.INFRA, 1.0),
                       (eis.Method.INFRA, 3.5))
]


@pytest.mark.parametrize("name,method,ws", WINDOW_CASES,
                         ids=[f"{n}-{eis.Method(m).name}-{w}" for n, m, w in WINDOW_CASES])
def test_window_bitmaps_equal_oracle(name, method, ws):
    if name not in G["windows"]:
        pytest.skip(f"{name}: not in oracle_windows.json (run make_oracle_goldens.py)")
    w = G["windows"][name]
    _say(f"{name} [{w['a']}, {w['b']}) method={eis.Method(method).name} window_scale={ws}")
    with eis.Context(method=method, window_scale=ws) as c:
        sq, eb, ns, ne = c.eis_classify(w["a"], w["b"])
    _check_window(name, sq, eb, ns, ne)


def test_mid_window_against_live_oracle():
    """The 10^9 window bit for bit against the oracle run here and now."""
    a, b = workloads.MID
    _say(f"live oracle on [{a}, {b})")
    t0 = time.perf_counter()
    ref = oracle.classify_range(a, b)
    _say(f"oracle took {time.perf_counter() - t0:.1f} s")
    with eis.Context(method=eis.Method.INFRA) as c:
        sq, eb, ns, ne = c.eis_classify(a, b)
    n = eis.eis_num_candidates(a, b)
    nb = (n + 7) // 8
    assert (ns, ne) == (ref["n_sqfree"], ref["n_eis"])
    assert np.array_equal(sq[:nb], ref["sq_bits"][:nb])
    assert np.array_equal(eb[:nb], ref["eis_bits"][:nb])
    _check_window("mid_1e9", sq, eb, ns, ne)


def test_async_device_pointers_on_table1_window():
    torch = pytest.importorskip("torch")
    if "table1_1e11" not in G["windows"]:
        pytest.skip("table1_1e11: not in oracle_windows.json (run make_oracle_goldens.py)")
    w = G["windows"]["table1_1e11"]
    nb = (w["n_cand"] + 7) // 8
    dev = torch.device("cuda:0")
    sq = torch.zeros(nb, dtype=torch.uint8, device=dev)
    eb = torch.zeros(nb, dtype=torch.uint8, device=dev)
    cnt = torch.zeros(2, dtype=torch.int64, device=dev)
    with eis.Context(method=eis.Method.AUTO) as c:
        st = torch.cuda.current_stream()
        c.eis_classify_async(w["a"], w["b"], sq.data_ptr(), eb.data_ptr(), cnt.data_ptr(),
                             st.cuda_stream)
        st.synchronize()
        assert c.eis_last_error() == 0
    _check_window("table1_1e11", sq.cpu().numpy(), eb.cpu().numpy(),
                  int(cnt[0].item()), int(cnt[1].item()))


def _tune_file(tmp_path, method_of_bin, ws_of_bin, chunk_of_bin=None, plog_of_bin=None):
    def shape(b):
        out = ""
        if chunk_of_bin:
            out += f', "walk_chunk": {chunk_of_bin(b)}'
        if plog_of_bin:
            out += f', "pass_log2": {plog_of_bin(b)}'
        return out
    bins = ",\n".join(
        f'  {{"b": {b}, "method": {method_of_bin(b)}, "window_scale": {ws_of_bin(b):.3f}{shape(b)}}}'
        for b in range(25))
    path = tmp_path / "tune.json"
    path.write_text('{"arch": "gfx950", "bins": [\n' + bins + "\n]}\n")
    return str(path)


def _batch(kind):
    rs = G[kind]["ranges"]
    return [r[0] for r in rs], [r[1] for r in rs], [(r[2], r[3]) for r in rs]


BATCH_CASES = [
    ("auto-graphs", dict(method=eis.Method.AUTO)),
    ("auto-nographs", dict(method=eis.Method.AUTO, flags=eis.EIS_FLAG_NO_GRAPHS)),
    ("infra-graphs", dict(method=eis.Method.INFRA)),
    ("infra-nographs", dict(method=eis.Method.INFRA, flags=eis.EIS_FLAG_NO_GRAPHS)),
    ("baby-graphs", dict(method=eis.Method.BABY)),
    ("infra-scale1", dict(method=eis.Method.INFRA, window_scale=1.0)),
    ("infra-scale5", dict(method=eis.Method.INFRA, window_scale=5.0)),
]


@pytest.mark.parametrize("label,kw", BATCH_CASES, ids=[c[0] for c in BATCH_CASES])
def test_batch_ranges_equal_oracle(label, kw):
    a, b, want = _batch("batch")
    _say(f"64 uneven ranges batched: {label}")
    with eis.Context(**kw) as c:
        for rep in range(2):  # the second call replays the captured graphs
            s, e = c.eis_count_batch(a, b)
            got = [(int(x), int(y)) for x, y in zip(s, e)]
            assert got == want, (label, rep)


def test_batch_ranges_tuned_mixed_choices(tmp_path):
    """A tuned context whose per-height choices alternate between the plain
    walk and giant steps at several window scales: one batch mixes all of
    them and must still equal the oracle."""
    scales = [1.0, 1.5, 1.75, 2.0, 2.25, 2.5, 3.5, 5.0]
    path = _tune_file(tmp_path, lambda b: (b % 3 != 0) * 1, lambda b: scales[b % len(scales)])
    a, b, want = _batch("batch")
    with eis.Context(tune_cache_path=path) as c:
        assert c.eis_tuned_choice(10**11)[0] in (eis.Method.BABY, eis.Method.INFRA)
        s, e = c.eis_count_batch(a, b)
        got = [(int(x), int(y)) for x, y in zip(s, e)]
        assert got == want
        # and one range at a time
        for k in (0, 17, 63):
            assert c.eis_count(a[k], b[k]) == want[k]


def test_serving_stream_equals_oracle():
    a, b, want = _batch("serve")
    reqs = workloads.serve_requests(len(a), G["serve"]["rate"])
    assert [(r[1], r[2]) for r in reqs] == list(zip(a, b))
    with eis.Context(serve_slots=64) as c:
        _say(f"serving {len(a)} requests open loop at {G['serve']['rate']} req/s")
        tickets = []
        t0 = time.perf_counter()
        for t_arr, x, y in reqs:
            now = time.perf_counter() - t0
            if t_arr > now:
                time.sleep(t_arr - now)
            tickets.append(c.eis_submit(x, y))
        got = [c.eis_wait(t, 60_000_000) for t in tickets]
    assert got == want
    with eis.Context() as c:
        s, e = c.eis_count_batch(a, b)
        assert [(int(x), int(y)) for x, y in zip(s, e)] == want


VARIANTS = [
    ("no-conjugate", eis.EIS_FLAG_NO_CONJUGATE_LOOKUPS),
    ("no-small-norm", eis.EIS_FLAG_NO_SMALL_NORM_PRODUCT),
    ("both", eis.EIS_FLAG_NO_CONJUGATE_LOOKUPS | eis.EIS_FLAG_NO_SMALL_NORM_PRODUCT),
]


@pytest.mark.parametrize("label,flags", VARIANTS, ids=[v[0] for v in VARIANTS])
def test_method_variants_give_the_same_bits(label, flags):
    """The switchable variants of the giant-step method (the paper's stride
    with direct lookups only; NUCOMP with partial reduction for small norms
    too) against the oracle: the plain-walk slice [5, 10^6] bit for bit with
    the live oracle, and the 10^9 and Table 1 windows against the goldens."""
    a, b = workloads.SMALL
    ref = oracle.classify_range(a, b)
    with eis.Context(method=eis.Method.INFRA, flags=flags) as c:
        sq, eb, ns, ne = c.eis_classify(a, b)
        n = eis.eis_num_candidates(a, b)
        nb = (n + 7) // 8
        assert (ns, ne) == (ref["n_sqfree"], ref["n_eis"])
        assert np.array_equal(eb[:nb], ref["eis_bits"][:nb])
        for name in ("mid_1e9", "table1_1e11"):
            if name not in G["windows"]:
                continue
            w = G["windows"][name]
            s0 = c.eis_get_stats()
            sq, eb, ns, ne = c.eis_classify(w["a"], w["b"])
            s1 = c.eis_get_stats()
            _say(f"{label} {name}: giant steps {s1['giant_steps'] - s0['giant_steps']}, "
                 f"retried {s1['giant_retries'] - s0['giant_retries']}, "
                 f"to the plain walk {s1['fallbacks'] - s0['fallbacks']}")
            _check_window(name, sq, eb, ns, ne)


def test_tuned_shape_knobs_give_the_same_bits(tmp_path):
    """Every tuned shape parameter -- the giant walk's walk chunk (8, 16, 32
    reduction steps per phase) and the pass size a range is cut into (2^22,
    2^23, 2^24 candidates) -- with the giant-step method at several scales:
    the full windows and the 64-range batch equal the oracle's goldens."""
    chunks, plogs, scales = [8, 16, 32], [22, 23, 24], [1.5, 2.0, 3.5]
    path = _tune_file(tmp_path, lambda b: 1 if b >= 12 else 0, lambda b: scales[b % 3],
                      lambda b: chunks[b % 3], lambda b: plogs[(b // 3) % 3])
    with eis.Context(tune_cache_path=path) as c:
        seen = {c.eis_tuned_shape(d) for d in (10**9, 4 * 10**9, 10**11 - 1, 10**12 - 1)}
        assert all(ch in chunks and ps in (2**22, 2**23, 2**24) for ch, ps in seen)
        assert len(seen) > 1
        for name in ("mid_1e9", "table1_1e11", "top_1e12"):
            if name not in G["windows"]:
                continue
            w = G["windows"][name]
            _say(f"tuned shapes {c.eis_tuned_shape(w['a'])} on {name}")
            sq, eb, ns, ne = c.eis_classify(w["a"], w["b"])
            _check_window(name, sq, eb, ns, ne)
        a, b, want = _batch("batch")
        s, e = c.eis_count_batch(a, b)
        assert [(int(x), int(y)) for x, y in zip(s, e)] == want
