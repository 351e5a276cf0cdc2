"""Seeded synthetic workloads (integer ranges).  No arithmetic of the method.

The paper sweeps every d <= 10^11; these ranges are slices of that sweep at
the same heights, generated from a recorded seed where they are random.
Both the GPU path and the oracle receive the same ranges from here.
"""
from __future__ import annotations

import numpy as np

# Plain baby-step slice: 5 <= d <= 10^6.
SMALL = (5, 10**6 + 1)
# Plain vs infrastructure: d in [10^9, 10^9 + 10^7).
MID = (10**9, 10**9 + 10**7)
# Large height, the last 10^8-window below 10^11 (also a window of Table 1).
LARGE = (10**11 - 10**8, 10**11)

BATCH_SEED = 20250709
SERVE_SEED = 20250710


def batch_ranges(n: int = 64, seed: int = BATCH_SEED):
    """Uneven ranges: start heights log-uniform in [10^6, 10^11], widths
    log-uniform in [10^4, 10^7]."""
    rng = np.random.default_rng(seed)
    a = np.floor(10.0 ** rng.uniform(6, 11, size=n)).astype(np.int64)
    w = np.floor(10.0 ** rng.uniform(4, 7, size=n)).astype(np.int64)
    b = np.minimum(a + w, 10**11)
    return [(int(x), int(y)) for x, y in zip(a, b)]


def serve_requests(n: int, rate: float, seed: int = SERVE_SEED):
    """Open-loop Poisson arrivals at `rate` req/s: list of (t_arrival_s, a, b),
    a log-uniform in [10^6, 10^11], width log-uniform in [10^3, 10^7]."""
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate, size=n)
    t = np.cumsum(gaps) - gaps[0]
    a = np.floor(10.0 ** rng.uniform(6, 11, size=n)).astype(np.int64)
    w = np.floor(10.0 ** rng.uniform(3, 7, size=n)).astype(np.int64)
    b = np.minimum(a + w, 10**11)
    return [(float(ti), int(x), int(y)) for ti, x, y in zip(t, a, b)]


def sample_indices(n_cand: int, k: int, seed: int):
    """k distinct candidate indices in [0, n_cand), sorted."""
    rng = np.random.default_rng(seed)
    k = min(k, n_cand)
    return np.sort(rng.choice(n_cand, size=k, replace=False))
