"""GPU tests against a closed form: the Richaud-Degert families d = n^2 +- 4.

For n odd, u = (n + sqrt d)/2 is a unit of norm -+1 and u = (n - 1)/2 + omega
(omega = (1 + sqrt d)/2) is not 1 mod 2 O_K; u is a positive power of the
fundamental unit, so that is not 1 mod 2 O_K either.  No member of D of
these forms is in E, at any height.  Their periods are a few steps long, so
at large heights they leave the walks at the half-period exit long before
the window ends: an edge case of both methods, checked here without the
oracle.  The sampled n run from 10^3 to 10^6 (d up to 10^12).
"""
import sys

import numpy as np
import pytest

import paper_2507_06579_amd as eis

pytestmark = pytest.mark.gpu


def _say(msg):
    print(f"[gpu-families] {msg}", flush=True)
    sys.stdout.flush()


def _family_members():
    ns = np.unique(np.round(np.logspace(3, 6, 400)).astype(np.int64) | 1)
    ds = [int(n) * int(n) + 4 for n in ns] + [int(n) * int(n) - 4 for n in ns]
    return sorted(d for d in ds if 5 <= d < eis.EIS_MAX_D)


@pytest.mark.parametrize("method", [eis.Method.BABY, eis.Method.INFRA])
def test_richaud_degert_members_are_not_eisenstein(method):
    ds = _family_members()
    _say(f"{len(ds)} single-candidate ranges, method {eis.Method(method).name}")
    with eis.Context(method=method) as c:
        n_sq, n_e = c.eis_count_batch(ds, [d + 1 for d in ds])
    assert int(n_e.sum()) == 0
    # the sieve finds the squarefree ones (about 8/pi^2 of them)
    assert 0.6 * len(ds) < int(n_sq.sum()) <= len(ds)
    # one classify call at the top of the range, bit by bit
    d = ds[-1]
    with eis.Context(method=method) as c:
        sq, eb, ns, ne = c.eis_classify(d, d + 1)
    assert ne == 0 and not np.asarray(eb).any()
