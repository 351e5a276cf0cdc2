"""GPU test of eis_classify_async_noalloc, the entry point that allocates
nothing (its kernels work in a fixed device scratch).

Its outputs must equal eis_classify_async's on the same ranges, bit for bit,
on two calls in a row -- the second with a smaller range, so that leftovers
of the first call in the shared scratch would show -- at heights where the
plain walk runs and where giant steps run in several scratch-sized batches.
"""
import sys

import numpy as np
import pytest

import paper_2507_06579_amd as eis

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _say(msg):
    print(f"[gpu-noalloc] {msg}", flush=True)
    sys.stdout.flush()


def _run(c, fn, a, b):
    n = eis.eis_num_candidates(a, b)
    nb = max(1, (n + 7) // 8)
    dev = torch.device("cuda:0")
    # poison the outputs so that a byte left unwritten shows
    sq = torch.full((nb + 8,), 0xA5, dtype=torch.uint8, device=dev)
    eb = torch.full((nb + 8,), 0x5A, dtype=torch.uint8, device=dev)
    cnt = torch.full((2,), -1, dtype=torch.int64, device=dev)
    st = torch.cuda.current_stream()
    getattr(c, fn)(a, b, sq.data_ptr(), eb.data_ptr(), cnt.data_ptr(), st.cuda_stream)
    st.synchronize()
    assert c.eis_last_error() == 0
    return (sq.cpu().numpy(), eb.cpu().numpy(), int(cnt[0].item()), int(cnt[1].item()), nb)


# (first range, second smaller range, method)
CASES = [
    ((10**9, 10**9 + 8 * 2**20), (10**9 + 5000, 10**9 + 5000 + 8 * 70001), eis.Method.BABY),
    ((10**11 - 8 * 2**20, 10**11), (10**11 - 8 * 300001 - 13, 10**11 - 13), eis.Method.INFRA),
    ((10**12 - 8 * 2**20, 10**12), (10**12 - 8 * 123457, 10**12 - 3), eis.Method.AUTO),
    ((10**6, 10**6 + 8 * 2**19 + 3), (5, 5000), eis.Method.AUTO),
]


@pytest.mark.parametrize("r1,r2,method", CASES, ids=["plain-1e9", "giant-1e11", "auto-1e12",
                                                   "small"])
def test_noalloc_equals_async_twice(r1, r2, method):
    with eis.Context(method=method) as c:
        for a, b in (r1, r2):
            _say(f"[{a}, {b}) method={eis.Method(method).name}")
            ref = _run(c, "eis_classify_async", a, b)
            got = _run(c, "eis_classify_async_noalloc", a, b)
            nb = ref[4]
            assert (got[2], got[3]) == (ref[2], ref[3])
            assert np.array_equal(got[0][:nb], ref[0][:nb])
            assert np.array_equal(got[1][:nb], ref[1][:nb])
            # nothing written past the bitmaps
            assert (got[0][nb:] == 0xA5).all() and (got[1][nb:] == 0x5A).all()


def test_noalloc_rejects_too_large_and_handles_empty():
    with eis.Context() as c:
        a = 10**10
        b = a + 8 * eis.NOALLOC_MAX_CANDIDATES + 8
        with pytest.raises(eis.EisError) as ei:
            c.eis_classify_async_noalloc(a, b, 0, 0, 0)
        assert ei.value.status == eis.Status.ENOMEM
        got = _run(c, "eis_classify_async_noalloc", 100, 100)
        assert (got[2], got[3]) == (0, 0)
        with pytest.raises(eis.EisError) as ei:
            c.eis_classify_async_noalloc(10, eis.EIS_MAX_D + 1, 0, 0, 0)
        assert ei.value.status == eis.Status.ERANGE
