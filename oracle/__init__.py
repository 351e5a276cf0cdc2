"""Plain CPU oracle for Eisenstein discriminants -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  The product library never links,
loads or calls it, and the two share no code.

The arithmetic lives in ``eis_oracle.c`` (plain C, built with gcc into
``liboracle.so``); this module is argument marshalling through ctypes.  Every
function follows the definitions of the paper's Section 1 (the sets D and E,
the counting function pi_E) and the reduction map rho of Appendix A; see the
header comment of ``eis_oracle.c`` for the derivation.

Parity status of each function (what pins it, see tests/test_oracle.py):
  walk_mod2          pinned: Pell brute force, class-number ratio, Table 1
                     window count, worked Example 2.5, big-int agreement
  unit_bigint        pinned: norm x0^2 - d y0^2 = +-4, least Pell solution,
                     the textbook units of Q(sqrt 5), Q(sqrt 13), Q(sqrt 21)
  sqfree_range       pinned: trial division, Moebius count
  mobius_count       pinned: trial division on small ranges
  narrow_class_number pinned: tabulated class numbers of small discriminants
  pell_least_y       pinned: direct check of the returned solution
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "eis_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

_lib = None


def build(force: bool = True) -> str:
    """Compile ``liboracle.so`` with gcc (plain -O2, no vectorisation tricks)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        cmd = ["gcc", "-std=c11", "-O2", "-fPIC", "-shared", "-pthread",
               "-Wall", "-Wno-unused-function", "-o", tmp, _SRC]
        subprocess.check_call(cmd)
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB):
        build(force=True)
    L = ctypes.CDLL(_LIB)
    u64, i64, c_int = ctypes.c_uint64, ctypes.c_int64, ctypes.c_int
    P = ctypes.POINTER
    L.orc_isqrt.argtypes = [u64]; L.orc_isqrt.restype = u64
    L.orc_is_squarefree_trial.argtypes = [u64]; L.orc_is_squarefree_trial.restype = c_int
    L.orc_in_D_trial.argtypes = [u64]; L.orc_in_D_trial.restype = c_int
    L.orc_num_candidates.argtypes = [u64, u64]; L.orc_num_candidates.restype = u64
    L.orc_first_candidate.argtypes = [u64]; L.orc_first_candidate.restype = u64
    L.orc_sqfree_range.argtypes = [u64, u64, ctypes.c_void_p, ctypes.c_size_t]
    L.orc_sqfree_range.restype = i64
    L.orc_mobius_count.argtypes = [u64, u64]; L.orc_mobius_count.restype = i64
    L.orc_walk_mod2.argtypes = [u64, P(u64), P(c_int)]; L.orc_walk_mod2.restype = c_int
    L.orc_unit_bigint.argtypes = [u64, ctypes.c_char_p, ctypes.c_char_p, ctypes.c_size_t,
                                  P(c_int), P(u64), P(u64)]
    L.orc_unit_bigint.restype = c_int
    L.orc_pell_least_y.argtypes = [u64, u64, P(u64), P(c_int)]
    L.orc_pell_least_y.restype = u64
    L.orc_narrow_class_number.argtypes = [i64]; L.orc_narrow_class_number.restype = i64
    L.orc_classify_range.argtypes = [u64, u64, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t,
                                     P(u64), P(u64), c_int, P(u64)]
    L.orc_classify_range.restype = c_int
    L.orc_classify_list.argtypes = [ctypes.c_void_p, u64, ctypes.c_void_p, c_int, P(u64)]
    L.orc_classify_list.restype = c_int
    L.orc_set_mutation.argtypes = [c_int]; L.orc_set_mutation.restype = None
    L.orc_is_prime_trial.argtypes = [u64]; L.orc_is_prime_trial.restype = c_int
    L.orc_count_primes_trial.argtypes = [u64, u64]; L.orc_count_primes_trial.restype = u64
    _lib = L
    return L


def isqrt(n: int) -> int:
    return int(_load().orc_isqrt(n))


def is_squarefree_trial(d: int) -> bool:
    return bool(_load().orc_is_squarefree_trial(d))


def in_D_trial(d: int) -> bool:
    return bool(_load().orc_in_D_trial(d))


def num_candidates(a: int, b: int) -> int:
    return int(_load().orc_num_candidates(a, b))


def first_candidate(a: int) -> int:
    return int(_load().orc_first_candidate(a))


def nbytes_for(a: int, b: int) -> int:
    return (num_candidates(a, b) + 7) // 8


def sqfree_range(a: int, b: int):
    """(bitmap uint8 array, count) of D over the candidates of [a, b)."""
    nb = max(1, nbytes_for(a, b))
    buf = np.zeros(nb, dtype=np.uint8)
    c = _load().orc_sqfree_range(a, b, buf.ctypes.data, nb)
    if c < 0:
        raise RuntimeError("orc_sqfree_range failed")
    return buf, int(c)


def mobius_count(a: int, b: int) -> int:
    return int(_load().orc_mobius_count(a, b))


def walk_mod2(d: int):
    """(flag, period l, Z/3 log-sum S_l) of the full CF period of (1+sqrt d)/2."""
    l = ctypes.c_uint64(0)
    S = ctypes.c_int(0)
    f = _load().orc_walk_mod2(d, ctypes.byref(l), ctypes.byref(S))
    if f < 0:
        raise RuntimeError(f"orc_walk_mod2 failed for d={d}")
    return bool(f), int(l.value), int(S.value)


def unit_bigint(d: int, cap: int = 1 << 16):
    """(flag, x0, y0, norm_sign, period) with eps_d = (x0 + y0 sqrt d)/2.

    x0 and y0 are Python ints when their decimal form fits ``cap`` characters
    and has at most 4000 digits, else None (the flag and norm check are still
    exact)."""
    xb = ctypes.create_string_buffer(cap)
    yb = ctypes.create_string_buffer(cap)
    sign = ctypes.c_int(0)
    l = ctypes.c_uint64(0)
    bits = ctypes.c_uint64(0)
    f = _load().orc_unit_bigint(d, xb, yb, cap, ctypes.byref(sign), ctypes.byref(l),
                                ctypes.byref(bits))
    if f < 0:
        raise RuntimeError(f"orc_unit_bigint failed for d={d}")
    x0 = int(xb.value) if 0 < len(xb.value) <= 4000 else None
    y0 = int(yb.value) if 0 < len(yb.value) <= 4000 else None
    return bool(f), x0, y0, int(sign.value), int(l.value)


def pell_least_y(d: int, ymax: int):
    """Least y <= ymax with d*y^2 +- 4 a square: (y, x, sign) or None."""
    x = ctypes.c_uint64(0)
    s = ctypes.c_int(0)
    y = _load().orc_pell_least_y(d, ymax, ctypes.byref(x), ctypes.byref(s))
    if y == 0:
        return None
    return int(y), int(x.value), int(s.value)


def narrow_class_number(D: int) -> int:
    h = int(_load().orc_narrow_class_number(D))
    if h < 0:
        raise RuntimeError(f"orc_narrow_class_number failed for D={D}")
    return h


def classify_range(a: int, b: int, nthreads: int | None = None, want_bits: bool = True):
    """Classify [a, b).  Returns dict(sq_bits, eis_bits, n_sqfree, n_eis, steps)."""
    if nthreads is None:
        nthreads = os.cpu_count() or 1
    nb = max(1, nbytes_for(a, b))
    sq = np.zeros(nb, dtype=np.uint8) if want_bits else None
    eb = np.zeros(nb, dtype=np.uint8) if want_bits else None
    nsq = ctypes.c_uint64(0)
    ne = ctypes.c_uint64(0)
    steps = ctypes.c_uint64(0)
    rc = _load().orc_classify_range(
        a, b, sq.ctypes.data if sq is not None else None,
        eb.ctypes.data if eb is not None else None, nb,
        ctypes.byref(nsq), ctypes.byref(ne), int(nthreads), ctypes.byref(steps))
    if rc != 0:
        raise RuntimeError("orc_classify_range failed")
    return dict(sq_bits=sq, eis_bits=eb, n_sqfree=int(nsq.value), n_eis=int(ne.value),
                steps=int(steps.value))


def is_prime_trial(n: int) -> bool:
    return bool(_load().orc_is_prime_trial(n))


def count_primes_trial(lo: int, hi: int) -> int:
    """Number of primes in [lo, hi) by trial division."""
    return int(_load().orc_count_primes_trial(lo, hi))


def classify_primes(a: int, b: int, nthreads: int | None = None):
    """The prime subsequence of [a, b) (Section 3.2): primes p = 5 (mod 8),
    found by trial division, and how many of them lie in E (the full-period
    walk).  Returns (n_primes, n_eis)."""
    d0 = first_candidate(a)
    ps = [d for d in range(d0, b, 8) if is_prime_trial(d)]
    if not ps:
        return 0, 0
    flags, _ = classify_list(ps, nthreads)
    return len(ps), int(flags.sum())


def classify_list(ds, nthreads: int | None = None):
    """Eisenstein flags (uint8 array) for an explicit list of members of D."""
    if nthreads is None:
        nthreads = os.cpu_count() or 1
    arr = np.ascontiguousarray(np.asarray(ds, dtype=np.uint64))
    flags = np.zeros(max(1, arr.size), dtype=np.uint8)
    steps = ctypes.c_uint64(0)
    rc = _load().orc_classify_list(arr.ctypes.data, arr.size, flags.ctypes.data,
                                   int(nthreads), ctypes.byref(steps))
    if rc != 0:
        raise RuntimeError("orc_classify_list failed")
    return flags[:arr.size], int(steps.value)


class mutation:
    """Context manager that plants a known mistake in the oracle (tests only)."""

    def __init__(self, which: int):
        self.which = which

    def __enter__(self):
        _load().orc_set_mutation(self.which)
        return self

    def __exit__(self, *exc):
        _load().orc_set_mutation(0)
        return False
