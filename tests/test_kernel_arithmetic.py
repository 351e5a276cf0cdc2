"""Host checks of the arithmetic facts the giant-step and window kernels rely
on, each restated here from its stated reasoning and checked by exhaustion or
on random inputs, with the device's fp32 reciprocal modelled as the correctly
rounded one or one ulp off either way.  No GPU is used.

* the byte-parallel fingerprint match of a table group (eis_infra.hip,
  group_match, group_entry, group_open);
* the extended Euclid with nearest-integer quotients (eis_giant.h, xgcd1):
  termination, the gcd, the cofactor class and its bound;
* the partial Euclid's floor quotient without correction below 2^21 / 1.5
  (eis_giant.h, neg_fl_div32);
* NUCOMP's gcd branch (Appendix A, NUCOMP): B_x mod B_y does not depend on
  which Bezout cofactor b is used.
"""
import math
import random

import numpy as np
import pytest

F32 = np.float32


def rcp32(b, mode):
    """fp32 reciprocal: correctly rounded (mode 0) or one ulp below / above."""
    r = (F32(1.0) / b).astype(F32)
    if mode == 1:
        r = np.nextafter(r, F32(0.0)).astype(F32)
    elif mode == 2:
        r = np.nextafter(r, F32(np.inf)).astype(F32)
    return r


# ---------------------------------------------------------------------------
# byte-parallel fingerprint match


def _differs(w, pat):
    x = (w ^ pat) & 0xFFFFFFFF
    return (((x & 0x7E007E00) + 0x7E007E00) | x) & 0xFFFFFFFF


def _perm(s0, s1, sel):
    """v_perm_b32: result byte i = byte sel_i of the 64-bit {s0 (high), s1 (low)}."""
    v = (np.uint64(s0) << np.uint64(32)) | np.uint64(s1)
    r = 0
    for i in range(4):
        b = (sel >> (8 * i)) & 0xFF
        r |= int((v >> np.uint64(8 * b)) & np.uint64(0xFF)) << (8 * i)
    return r


def test_fingerprint_field_test_is_exact():
    # every 16-bit field value against every nonzero 7-bit fingerprint, in
    # both halves of a word: bit 15 (31) of the expression is set iff the
    # field's bits 9-15 differ from the fingerprint
    v = np.arange(1 << 16, dtype=np.uint64)
    for fp in range(1, 128):
        f = fp << 9
        pat = np.uint64(f | (f << 16))
        lo = _differs(v, pat)
        assert np.array_equal(((lo >> np.uint64(15)) & np.uint64(1)) == 0, (v >> np.uint64(9)) == fp)
        hi = _differs(v << np.uint64(16), pat)
        assert np.array_equal(((hi >> np.uint64(31)) & np.uint64(1)) == 0, (v >> np.uint64(9)) == fp)
        # the low field's sum never carries into the high field
        mixed = _differs(v | (np.uint64(0x1FF) << np.uint64(16)) | (np.uint64(fp) << np.uint64(25)), pat)
        assert np.all(((mixed >> np.uint64(31)) & np.uint64(1)) == 0)


def _group_match(g, f):
    pat = f | (f << 16)
    lo = _perm(_differs(g[1], pat), _differs(g[0], pat), 0x07050301)
    hi = _perm(_differs(g[3], pat), _differs(g[2], pat), 0x07050301)
    return ~((hi << 32) | lo) & 0x8080808080808080


def _group_entry(g, bit):
    h = ((g[3] << 32) | g[2]) if bit >= 32 else ((g[1] << 32) | g[0])
    return ((h >> ((bit << 1) & 0x30)) & 0x1FF) - 1


def test_group_match_entry_and_open():
    rng = random.Random(20250709)
    for _ in range(20000):
        fp = rng.randrange(1, 128)
        fill = rng.randrange(0, 9)
        slots = []
        for i in range(8):
            if i < fill:
                p = fp if rng.random() < 0.3 else rng.randrange(1, 128)
                slots.append((p << 9) | rng.randrange(1, 512))
            else:
                slots.append(0)  # a group fills its first slots
        g = [slots[2 * k] | (slots[2 * k + 1] << 16) for k in range(4)]
        m = _group_match(g, fp << 9)
        want = [i for i in range(8) if slots[i] and slots[i] >> 9 == fp]
        got = [i for i in range(8) if (m >> (8 * i + 7)) & 1]
        assert got == want
        assert m & ~0x8080808080808080 == 0
        for i in want:
            assert _group_entry(g, 8 * i + 7) == (slots[i] & 0x1FF) - 1
        # an empty slot exists iff the last one is empty
        assert (g[3] < 0x10000) == (fill < 8)


# ---------------------------------------------------------------------------
# extended Euclid with nearest-integer quotients


def _xgcd_near(a0, b0, mode):
    """Vectorized fp32 restatement of the device loop on |a|, |b|; returns
    (g, x, iterations) with x A = g (mod B)."""
    a = np.abs(a0).astype(F32)
    b = np.abs(b0).astype(F32)
    x0 = np.ones_like(a)
    x1 = np.zeros_like(a)
    iters = np.zeros(a.shape, dtype=np.int64)
    for _ in range(64):
        run = (a != 0) & (b != 0)
        if not run.any():
            break
        q = np.rint((a * rcp32(np.where(run, b, F32(1)), mode)).astype(F32))
        na = (a - q * b).astype(F32)
        nx0 = (x0 - q * x1).astype(F32)
        a = np.where(run, na, a)
        x0 = np.where(run, nx0, x0)
        go = run & (a != 0)
        q = np.rint((b * rcp32(np.where(go, a, F32(1)), mode)).astype(F32))
        nb = (b - q * a).astype(F32)
        nx1 = (x1 - q * x0).astype(F32)
        b = np.where(go, nb, b)
        x1 = np.where(go, nx1, x1)
        iters += run
    assert not ((a != 0) & (b != 0)).any(), "did not terminate"
    az = a == 0
    gs = np.where(az, b, a)
    xs = np.where(az, x1, x0)
    return np.abs(gs).astype(np.int64), np.where(gs < 0, -xs, xs).astype(np.int64), iters


@pytest.mark.parametrize("mode", [0, 1, 2])
def test_nearest_integer_xgcd(mode):
    rng = np.random.default_rng(7 + mode)
    n = 200000
    A = rng.integers(0, 1 << 21, n)
    B = rng.integers(0, 1 << 21, n)
    k = rng.integers(1, 60, n // 4)  # pairs with a common factor
    A[: n // 4] = (A[: n // 4] // 64) * k
    B[: n // 4] = (B[: n // 4] // 64) * k
    g, x, iters = _xgcd_near(A, B, mode)
    ref = np.gcd(A, B)
    assert np.array_equal(g, ref)
    assert iters.max() <= 16
    ok = B > 0
    # x A = g (mod B), |x| <= B / g
    assert np.all(((x[ok] * A[ok] - g[ok]) % B[ok]) == 0)
    assert np.all(np.abs(x[ok]) * g[ok] <= B[ok])
    # the same class modulo B / g as the floor-quotient cofactor
    for i in np.flatnonzero(ok)[:3000]:
        a, b = int(A[i]), int(B[i])
        x0, x1, r0, r1 = 1, 0, a, b
        while r1:
            q = r0 // r1
            r0, r1, x0, x1 = r1, r0 - q * r1, x1, x0 - q * x1
        m = b // r0
        assert (x0 - int(x[i])) % m == 0


# ---------------------------------------------------------------------------
# partial Euclid: the biased floor quotient is exact below 2^21 / 1.5


@pytest.mark.parametrize("mode", [0, 1, 2])
def test_biased_floor_quotient_below_bound(mode):
    rng = np.random.default_rng(11 + mode)
    n = 400000
    a = rng.integers(0, 1398102, n)
    b = np.maximum(1, (a / rng.uniform(1.0, 3000.0, n)).astype(np.int64))
    b[: n // 8] = rng.integers(1, 64, n // 8)
    # quotients just below and at integers: a = k b - 1 and a = k b
    k = rng.integers(1, 1000, n // 8)
    bb = rng.integers(1, 1398, n // 8)
    a[n // 8: n // 4] = np.minimum(k * bb - 1, 1398101)
    b[n // 8: n // 4] = bb
    a[n // 4: 3 * n // 8] = np.minimum(k * bb, 1398101)
    b[n // 4: 3 * n // 8] = bb
    af, bf = a.astype(F32), b.astype(F32)
    bias = F32(1.0) + F32(2.0 ** -21)
    nq = np.ceil((-(af * bias).astype(F32) * rcp32(bf, mode)).astype(F32))
    assert np.array_equal(-nq.astype(np.int64), a // b)


# ---------------------------------------------------------------------------
# NUCOMP's gcd branch does not depend on the Bezout cofactor's representative


def _egcd(a, b):
    x0, x1 = 1, 0
    while b:
        q = a // b
        a, b, x0, x1 = b, a - q * b, x1, x0 - q * x1
    return a, x0


def test_nucomp_gcd_branch_cofactor_class():
    rng = random.Random(3)
    D = 5 + 8 * 12345678901
    tested = 0
    while tested < 1000:
        def form():
            # (u, v, w) with v^2 - 4 u w = D, |v| <= u
            while True:
                u = rng.randrange(3, 400)
                v = rng.randrange(-u, u)
                if (v * v - D) % (4 * u) == 0:
                    return u, v, (v * v - D) // (4 * u)
        (u1, v1, w1), (u2, v2, w2) = form(), form()
        if w1 < w2:
            (u1, v1, w1), (u2, v2, w2) = (u2, v2, w2), (u1, v1, w1)
        if (v1 + v2) % 2:
            continue
        s = (v1 + v2) // 2
        m = v2 - s
        F, b0 = _egcd(u2, u1)
        if s % F == 0:
            continue
        G, y2 = _egcd(s % F, F)
        H, By = F // G, u1 // G
        seen = set()
        for k in range(-3, 4):
            b = b0 + k * (u1 // F)
            c = (F - b * u2) // u1
            assert b * u2 + c * u1 == F
            l = (y2 % H) * (((b % H) * (w1 % H) + (c % H) * (w2 % H)) % H) % H
            num = l * By + b * m
            assert num % H == 0
            seen.add((num // H) % By)
        assert len(seen) == 1
        tested += 1
    assert math.isfinite(tested)


# ---------------------------------------------------------------------------
# the reduction step's quotient (eis_walk.h, rho_step_q) needs no overshoot
# test for d <= 1.45 10^11, where s <= 380,788 and t = P + s < 2^24 / 13


@pytest.mark.parametrize("mode", [0, 1, 2])
def test_rho_quotient_exact_below_bound(mode):
    rng = np.random.default_rng(23 + mode)
    n = 400000
    s = rng.integers(100000, 380789, n)
    P = rng.integers(1, s + 1)
    # reduced: s - P < Q <= s + P; a third of the Q divide P + s exactly
    # and a third divide P + s + 1, so that t / Q sits at or just below an
    # integer
    lo, hi = s - P + 1, s + P
    Q = rng.integers(lo, hi + 1)
    t = P + s
    for part, off in ((1, 0), (2, 1)):
        sl = slice(part * n // 3, (part + 1) * n // 3)
        k = np.maximum(1, (t[sl] + off) // np.maximum(lo[sl], 1))
        q = (t[sl] + off) // k
        ok = (q >= lo[sl]) & (q <= hi[sl]) & ((t[sl] + off) % np.maximum(q, 1) == 0)
        Q[sl] = np.where(ok, q, Q[sl])
    c = 1.0 + 2.0 ** -21
    P4, Q4, s4 = (P / 4.0).astype(F32), (Q / 4.0).astype(F32), (s / 4.0).astype(F32)
    sqc = (s4.astype(np.float64) * np.float64(F32(c))).astype(F32)
    num = (P4.astype(np.float64) * np.float64(F32(c)) + sqc.astype(np.float64)).astype(F32)  # one fma
    q = np.floor((num * rcp32(Q4, mode)).astype(F32)).astype(np.int64)
    assert np.array_equal(q, t // Q)
