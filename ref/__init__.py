"""The paper's method on the CPU -- TEST INFRASTRUCTURE ONLY.

Algorithm "Infrastructure" of Appendix A, modified to carry generators in
(O_K/2O_K)^* ~ Z/3, with the giant steps of Algorithms NUCOMP, NUDUPL and
NUCOMPchoose (and the ideal product for small norms), in exact int64 /
__int128 arithmetic, with the distance (natural log of each generator)
tracked beside every residue.  Written in plain C (``eis_method.c``) from the
paper; it shares no code with the HIP path or with ``oracle/``.

Only ``tests/`` and the CPU-baseline leg of ``bench.py`` may import this
package: it pins the method's arithmetic (per composition and per d) and is
the second CPU baseline (the method itself, next to the oracle's plain
definition).  The product library never loads it.

Parity status (tests/test_ref_method.py):
  compose        pinned: the result lies on the cycle of reduced principal
                 ideals at the distance and with the residue the algorithm
                 claims (against the plain walk's table); gamma a unit at 2
  classify       pinned: flags equal the oracle's; the unit found lies at
                 exactly one regulator (the plain walk's ln eps)
  cycle          pinned: its period and regulator against the oracle's
                 period and the fundamental unit's size
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "eis_method.c")
_LIB = os.path.join(_HERE, "libref.so")

_lib = None

PATHS = ("product", "nudupl", "nucomp")


def build(force: bool = True) -> str:
    """Compile ``libref.so`` with gcc."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        cmd = ["gcc", "-std=c11", "-O2", "-fPIC", "-shared", "-pthread", "-Wall", "-o", tmp,
               _SRC, "-lm"]
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
    i64, c_int, dbl = ctypes.c_int64, ctypes.c_int, ctypes.c_double
    P = ctypes.POINTER
    vp = ctypes.c_void_p
    L.ref_cycle.argtypes = [i64, vp, vp, vp, vp, ctypes.c_long, P(dbl)]
    L.ref_cycle.restype = ctypes.c_long
    L.ref_compose.argtypes = [i64, i64, i64, i64, i64, c_int, vp, vp, P(dbl)]
    L.ref_compose.restype = c_int
    L.ref_classify.argtypes = [i64, dbl, i64, vp, P(dbl)]
    L.ref_classify.restype = c_int
    L.ref_classify_list.argtypes = [vp, ctypes.c_size_t, dbl, vp, c_int]
    L.ref_classify_list.restype = ctypes.c_long
    L.ref_set_mutation.argtypes = [c_int]
    L.ref_set_mutation.restype = None
    _lib = L
    return L


def cycle(d: int, cap: int | None = None):
    """The cycle of reduced principal ideals of Q(sqrt d) from (1): dict with
    arrays Q, P (entry j is (theta_{j+1}) = [Q_j/2, (P_j + sqrt d)/2], entry
    0 being (1) as (2, P_1)), dist (ln theta_{j+1}), res (its residue in
    Z/3), the period l and the regulator R = ln eps."""
    if cap is None:
        cap = max(64, int(4 * math.sqrt(d)) + 64)
    Q = np.zeros(cap, dtype=np.int64)
    Pa = np.zeros(cap, dtype=np.int64)
    dist = np.zeros(cap, dtype=np.float64)
    res = np.zeros(cap, dtype=np.int32)
    R = ctypes.c_double(0.0)
    n = _load().ref_cycle(d, Q.ctypes.data, Pa.ctypes.data, dist.ctypes.data, res.ctypes.data,
                          cap, ctypes.byref(R))
    if n < 0:
        raise RuntimeError(f"ref_cycle failed for d={d}")
    return dict(Q=Q[:n], P=Pa[:n], dist=dist[:n], res=res[:n], period=int(n), R=float(R.value))


def compose(d: int, Q1: int, P1: int, Q2: int, P2: int, mode: int = 0):
    """NUCOMPchoose of two reduced ideals and the reduction after it:
    (Q, P) of the result, the path taken, the reduction steps, the distance
    shift -ln|gamma| + sum ln|psi|, the residue shift (-log gamma + sum r)
    mod 3, and the error bits (0 = every check passed).  mode 0 is
    NUCOMPchoose as printed; mode 1 sends every pair through NUCOMP, squares
    included, with an unbounded L when a norm is <= 50."""
    out = np.zeros(2, dtype=np.int64)
    info = np.zeros(3, dtype=np.int32)
    shift = ctypes.c_double(0.0)
    err = _load().ref_compose(d, Q1, P1, Q2, P2, mode, out.ctypes.data, info.ctypes.data,
                              ctypes.byref(shift))
    return dict(Q=int(out[0]), P=int(out[1]), path=PATHS[int(info[0])], steps=int(info[1]),
                res=int(info[2]), shift=float(shift.value), err=int(err))


def classify(d: int, c: float = 1.0, max_giants: int = 1 << 26):
    """Algorithm Infrastructure on d with window c d^(1/4): dict with the
    flag (d in E), the unit's distance as found, baby and giant steps, how it
    ended ('half' period in the window or dictionary 'hit') and the error
    bits."""
    st = np.zeros(4, dtype=np.int64)
    e = ctypes.c_double(0.0)
    f = _load().ref_classify(d, c, max_giants, st.ctypes.data, ctypes.byref(e))
    return dict(flag=bool(f > 0) if f >= 0 else None, eps_dist=float(e.value),
                baby=int(st[0]), giants=int(st[1]),
                end={1: "half", 2: "hit"}.get(int(st[2]), "none"), err=int(st[3]))


def classify_list(ds, c: float = 1.0, nthreads: int | None = None):
    """Flags (uint8) of many members of D on all cores, and the count of d's
    whose computation failed a check."""
    if nthreads is None:
        nthreads = os.cpu_count() or 1
    arr = np.ascontiguousarray(np.asarray(ds, dtype=np.int64))
    flags = np.zeros(max(1, arr.size), dtype=np.uint8)
    bad = _load().ref_classify_list(arr.ctypes.data, arr.size, c, flags.ctypes.data,
                                    int(nthreads))
    return flags[:arr.size], int(bad)


class mutation:
    """Context manager that plants a known mistake in the method (tests only)."""

    def __init__(self, which: int):
        self.which = which

    def __enter__(self):
        _load().ref_set_mutation(self.which)
        return self

    def __exit__(self, *exc):
        _load().ref_set_mutation(0)
        return False
