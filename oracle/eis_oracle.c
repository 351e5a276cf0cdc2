/*
 * eis_oracle.c -- plain, slow, obviously-correct CPU oracle for Eisenstein
 * discriminants (Breuer & Punch, "Quadratic units and cubic fields").
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library may link, load or
 * call this file.  It is used by tests/, by the smoke check and by the
 * cpu_baseline leg of the benchmark, and nowhere else.  It shares no code,
 * header, table or constant with the HIP path.
 *
 * What it computes (Section 1 of the paper):
 *   D = { d > 0 : d = 5 (mod 8), d squarefree }
 *   E = { d in D : eps_d = 1 (mod 2 O_K) }
 * with O_K = Z[(1+sqrt d)/2] and eps_d = (x0 + y0 sqrt d)/2 the fundamental
 * unit.  Since Z[sqrt d] = Z + 2 O_K, eps_d = 1 (mod 2 O_K) holds exactly
 * when eps_d lies in Z[sqrt d] (equivalence (1) <=> (3) of Lemma 1.1), i.e.
 * when x0 and y0 are both even.  The oracle therefore computes eps_d itself
 * (big-integer mode) or its coordinates modulo 2 (mod-2 mode) from the full
 * continued-fraction period of (1 + sqrt d)/2, using the reduction map rho
 * exactly as Appendix A defines it:
 *     q_j = floor((P_j + sqrt d)/Q_j),  P_{j+1} = q_j Q_j - P_j,
 *     Q_{j+1} = (d - P_{j+1}^2)/Q_j,    (P_0, Q_0) = (1, 2),
 * together with the convergent recurrences A_j = q_j A_{j-1} + A_{j-2},
 * B_j = q_j B_{j-1} + B_{j-2}, A_{-2} = 0, A_{-1} = 1, B_{-2} = 1, B_{-1} = 0,
 * and the generator form theta_{j+2} = (G_j + B_j sqrt d)/2 with
 * G_j = 2 A_j - B_j (Appendix A, the paragraph before Theorem A.1).  The
 * period l is the first index with Q_l = 2, where theta_{l+1} = eps_d, so
 * x0 = 2 A_{l-1} - B_{l-1} and y0 = B_{l-1}.
 *
 * No half-period shortcut, no giant steps, no blocking: every walk goes
 * around the whole period.  Reduction mod 2 commutes with the recurrences
 * because Z -> F_2 is a ring map, so mod-2 mode is exact.
 *
 * The Z/3 log-sum (Appendix A, the text after Theorem A.1: (O_K/2O_K)^* is
 * F_4^* ~ Z/3, and the walk may carry generators in Z/3) is computed beside
 * the plain result, as a second characterisation checked by the tests:
 * the relative generator (P_{j+1} + sqrt d)/Q_j reduces to log 1 when
 * P_{j+1} = 1 (mod 4) and to log 2 when P_{j+1} = 3 (mod 4).
 *
 * Independent pins, also plain:
 *   - squarefree test by trial division, and a range sieve over p^2;
 *   - the Moebius count of D in a range;
 *   - the least y >= 1 with d y^2 +- 4 a square (Lemma 1.1 (2));
 *   - the narrow class number h+(D) by counting rho-cycles of reduced
 *     indefinite forms (Lemma 1.1 (4) in its narrow form).
 *
 * All functions are re-entrant except orc_set_mutation, which is a test knob
 * that plants a known mistake so that the tests can show the pins catch it.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <pthread.h>
#include <time.h>

typedef unsigned __int128 u128;

/* ------------------------------------------------------------------ */
/* Mutation knob (tests only).  0 = correct oracle.                    */
/*   1: drop the A_{j-2}, B_{j-2} terms of the convergent recurrence   */
/*   2: x0 = 2A + B instead of 2A - B                                  */
/*   3: residue taken from P_j instead of P_{j+1} (index slip)        */
/*   4: flag taken from A_{l-1} instead of B_{l-1}                     */
/* ------------------------------------------------------------------ */
static volatile int g_mutation = 0;
void orc_set_mutation(int m) { g_mutation = m; }

/* Guard against runaway walks: no period below 2^40 comes close. */
#define ORC_MAX_STEPS 200000000ULL

/* ------------------------------------------------------------------ */
/* Integer square root: largest r with r*r <= n.                       */
/* ------------------------------------------------------------------ */
uint64_t orc_isqrt(uint64_t n)
{
    /* bit-by-bit method: plain and exact for every 64-bit n */
    uint64_t r = 0;
    uint64_t bit = (uint64_t)1 << 62;
    while (bit > n) bit >>= 2;
    while (bit != 0) {
        if (n >= r + bit) {
            n -= r + bit;
            r = (r >> 1) + bit;
        } else {
            r >>= 1;
        }
        bit >>= 2;
    }
    return r;
}

/* ------------------------------------------------------------------ */
/* Squarefree test by trial division (Section 1: the definition of D). */
/* ------------------------------------------------------------------ */
int orc_is_squarefree_trial(uint64_t d)
{
    if (d == 0) return 0;
    uint64_t n = d;
    for (uint64_t p = 2; p * p <= n; p++) {
        if (n % p == 0) {
            n /= p;
            if (n % p == 0) return 0;
        }
    }
    return 1;
}

int orc_in_D_trial(uint64_t d)
{
    return (d % 8 == 5) && orc_is_squarefree_trial(d);
}

/* ------------------------------------------------------------------ */
/* Primality by trial division (the definition of a prime), for the prime */
/* subsequence of Section 3.2.                                           */
/* ------------------------------------------------------------------ */
int orc_is_prime_trial(uint64_t n)
{
    if (n < 2) return 0;
    if (n < 4) return 1;
    if (n % 2 == 0) return 0;
    for (uint64_t p = 3; p * p <= n; p += 2)
        if (n % p == 0) return 0;
    return 1;
}

/* Number of primes n with lo <= n < hi, by trial division. */
uint64_t orc_count_primes_trial(uint64_t lo, uint64_t hi)
{
    uint64_t c = 0;
    for (uint64_t n = lo; n < hi; n++) c += (uint64_t)orc_is_prime_trial(n);
    return c;
}

/* Number of candidates d = 5 (mod 8) with a <= d < b. */
uint64_t orc_num_candidates(uint64_t a, uint64_t b)
{
    if (a >= b) return 0;
    /* d0 = least d >= a with d = 5 mod 8 */
    uint64_t d0 = a + ((5 + 8 - (a % 8)) % 8);
    if (d0 >= b) return 0;
    return (b - 1 - d0) / 8 + 1;
}

uint64_t orc_first_candidate(uint64_t a)
{
    return a + ((5 + 8 - (a % 8)) % 8);
}

/* Plain Eratosthenes: odd primes p <= lim, returned in a malloc'd array. */
static uint32_t *odd_primes_upto(uint64_t lim, size_t *count)
{
    *count = 0;
    if (lim < 3) return NULL;
    uint8_t *comp = (uint8_t *)calloc(lim + 1, 1);
    size_t n = 0;
    for (uint64_t i = 2; i <= lim; i++) {
        if (!comp[i]) {
            if (i > 2) n++;
            for (uint64_t j = i * i; j <= lim; j += i) comp[j] = 1;
        }
    }
    uint32_t *pr = (uint32_t *)malloc(sizeof(uint32_t) * (n ? n : 1));
    size_t k = 0;
    for (uint64_t i = 3; i <= lim; i++)
        if (!comp[i]) pr[k++] = (uint32_t)i;
    free(comp);
    *count = n;
    return pr;
}

/*
 * Squarefree bitmap of the candidates in [a, b) by striking multiples of p^2
 * for every odd prime p with p^2 < b.  Bit i (LSB first in byte i/8) stands
 * for d0 + 8 i.  Returns the number of set bits (pi_D over the range).
 */
int64_t orc_sqfree_range(uint64_t a, uint64_t b, uint8_t *bits, size_t nbytes)
{
    uint64_t n = orc_num_candidates(a, b);
    if (nbytes < (n + 7) / 8) return -1;
    memset(bits, 0, nbytes);
    if (n == 0) return 0;
    uint64_t d0 = orc_first_candidate(a);
    for (uint64_t i = 0; i < n; i++) bits[i / 8] |= (uint8_t)(1u << (i % 8));
    size_t np = 0;
    uint32_t *pr = odd_primes_upto(orc_isqrt(b - 1), &np);
    for (size_t t = 0; t < np; t++) {
        uint64_t m = (uint64_t)pr[t] * pr[t];
        uint64_t x = ((a + m - 1) / m) * m; /* first multiple of m >= a */
        for (; x < b; x += m) {
            if (x % 8 == 5) {
                uint64_t i = (x - d0) / 8;
                bits[i / 8] &= (uint8_t)~(1u << (i % 8));
            }
        }
    }
    free(pr);
    int64_t c = 0;
    for (uint64_t i = 0; i < n; i++) c += (bits[i / 8] >> (i % 8)) & 1;
    return c;
}

/*
 * Moebius count of D in [a, b):
 *   sum over odd m with m^2 <= b-1 of mu(m) * #{x in [a,b): x = 5 (8), m^2 | x}.
 * The inner set is one residue class modulo 8 m^2 (gcd(8, m^2) = 1).
 */
static int moebius(uint64_t m)
{
    int mu = 1;
    for (uint64_t p = 2; p * p <= m; p++) {
        if (m % p == 0) {
            m /= p;
            if (m % p == 0) return 0;
            mu = -mu;
        }
    }
    if (m > 1) mu = -mu;
    return mu;
}

/* #{x : lo <= x < hi, x = c (mod M)}, 0 <= c < M */
static uint64_t count_class(uint64_t lo, uint64_t hi, uint64_t c, uint64_t M)
{
    if (lo >= hi) return 0;
    /* number of x = c + kM, k >= 0, with x < hi, minus those with x < lo */
    uint64_t below_hi = (hi > c) ? (hi - 1 - c) / M + 1 : 0;
    uint64_t below_lo = (lo > c) ? (lo - 1 - c) / M + 1 : 0;
    return below_hi - below_lo;
}

int64_t orc_mobius_count(uint64_t a, uint64_t b)
{
    if (a >= b) return 0;
    int64_t total = 0;
    for (uint64_t m = 1; m * m <= b - 1; m += 2) {
        int mu = moebius(m);
        if (mu == 0) continue;
        uint64_t m2 = m * m;
        uint64_t c = 0;
        for (uint64_t t = 0; t < 8; t++) {
            if ((m2 * t) % 8 == 5) { c = m2 * t; break; }
        }
        total += mu * (int64_t)count_class(a, b, c, 8 * m2);
    }
    return total;
}

/* ------------------------------------------------------------------ */
/* Full-period walk, mod-2 mode.                                       */
/* ------------------------------------------------------------------ */
/*
 * Returns 1 if d is Eisenstein, 0 if not, -1 on an internal error (inexact
 * division, runaway walk, d not = 5 mod 8).  Squarefreeness is not checked
 * here.  *period gets l, *log_sum gets S_l = sum r(P_i) mod 3.
 */
int orc_walk_mod2(uint64_t d, uint64_t *period, int *log_sum)
{
    if (d % 8 != 5 || d >= ((uint64_t)1 << 62)) return -1;
    const uint64_t s = orc_isqrt(d);
    uint64_t P = 1, Q = 2;
    unsigned A2 = 0, A1 = 1, B2 = 1, B1 = 0; /* A_{j-2}, A_{j-1}, B_{j-2}, B_{j-1} mod 2 */
    int S = 0;
    uint64_t j = 0;
    const int mut = g_mutation;
    for (;;) {
        uint64_t q = (P + s) / Q; /* = floor((P + sqrt d)/Q) for Q > 0 */
        unsigned qb = (unsigned)(q & 1);
        unsigned A = (qb * A1 + (mut == 1 ? 0 : A2)) & 1;
        unsigned B = (qb * B1 + (mut == 1 ? 0 : B2)) & 1;
        uint64_t Pn = q * Q - P;
        uint64_t sq = Pn * Pn;
        if (sq >= d) return -1;
        if ((d - sq) % Q != 0) return -1;
        uint64_t Qn = (d - sq) / Q;
        int r = (((mut == 3 ? P : Pn) % 4) == 1) ? 1 : 2;
        S = (S + r) % 3;
        A2 = A1; A1 = A; B2 = B1; B1 = B;
        P = Pn; Q = Qn;
        j++;
        if (Q == 2) break;
        if (j > ORC_MAX_STEPS) return -1;
    }
    if (period) *period = j;
    if (log_sum) *log_sum = S;
    /* eps_d in Z[sqrt d] <=> y0 = B_{l-1} even (then x0 = 2A - B is even). */
    if (mut == 4) return A1 == 0;
    return B1 == 0;
}

/* ------------------------------------------------------------------ */
/* Minimal unsigned big integers (little-endian 32-bit limbs).         */
/* ------------------------------------------------------------------ */
typedef struct { uint32_t *v; size_t n, cap; } bn;

static void bn_init(bn *x) { x->v = NULL; x->n = 0; x->cap = 0; }
static void bn_free(bn *x) { free(x->v); bn_init(x); }
static void bn_reserve(bn *x, size_t cap)
{
    if (cap > x->cap) {
        size_t nc = x->cap ? x->cap : 4;
        while (nc < cap) nc *= 2;
        x->v = (uint32_t *)realloc(x->v, nc * sizeof(uint32_t));
        x->cap = nc;
    }
}
static void bn_trim(bn *x) { while (x->n && x->v[x->n - 1] == 0) x->n--; }
static void bn_set_u64(bn *x, uint64_t a)
{
    bn_reserve(x, 2);
    x->v[0] = (uint32_t)a; x->v[1] = (uint32_t)(a >> 32); x->n = 2;
    bn_trim(x);
}
static void bn_copy(bn *dst, const bn *src)
{
    bn_reserve(dst, src->n + 1);
    if (src->n) memcpy(dst->v, src->v, src->n * sizeof(uint32_t));
    dst->n = src->n;
}
static int bn_cmp(const bn *a, const bn *b)
{
    if (a->n != b->n) return a->n < b->n ? -1 : 1;
    for (size_t i = a->n; i-- > 0;)
        if (a->v[i] != b->v[i]) return a->v[i] < b->v[i] ? -1 : 1;
    return 0;
}
/* r = a*q + c, q < 2^32; r may alias c but not a */
static void bn_mul_small_add(bn *r, const bn *a, uint32_t q, const bn *c)
{
    size_t n = (a->n > c->n ? a->n : c->n) + 1;
    uint32_t *out = (uint32_t *)calloc(n, sizeof(uint32_t));
    uint64_t carry = 0;
    for (size_t i = 0; i < n; i++) {
        uint64_t t = carry;
        if (i < a->n) t += (uint64_t)a->v[i] * q;
        if (i < c->n) t += c->v[i];
        out[i] = (uint32_t)t;
        carry = t >> 32;
    }
    free(r->v);
    r->v = out; r->n = n; r->cap = n;
    bn_trim(r);
}
/* r = a + b */
static void bn_add(bn *r, const bn *a, const bn *b)
{
    size_t n = (a->n > b->n ? a->n : b->n) + 1;
    uint32_t *out = (uint32_t *)calloc(n, sizeof(uint32_t));
    uint64_t carry = 0;
    for (size_t i = 0; i < n; i++) {
        uint64_t t = carry;
        if (i < a->n) t += a->v[i];
        if (i < b->n) t += b->v[i];
        out[i] = (uint32_t)t;
        carry = t >> 32;
    }
    free(r->v);
    r->v = out; r->n = n; r->cap = n;
    bn_trim(r);
}
/* r = a - b, requires a >= b */
static void bn_sub(bn *r, const bn *a, const bn *b)
{
    size_t n = a->n;
    uint32_t *out = (uint32_t *)calloc(n + 1, sizeof(uint32_t));
    int64_t borrow = 0;
    for (size_t i = 0; i < n; i++) {
        int64_t t = (int64_t)a->v[i] - borrow - (i < b->n ? (int64_t)b->v[i] : 0);
        if (t < 0) { t += ((int64_t)1 << 32); borrow = 1; } else borrow = 0;
        out[i] = (uint32_t)t;
    }
    free(r->v);
    r->v = out; r->n = n; r->cap = n + 1;
    bn_trim(r);
}
/* r = a*b, schoolbook */
static void bn_mul(bn *r, const bn *a, const bn *b)
{
    size_t n = a->n + b->n + 1;
    uint32_t *out = (uint32_t *)calloc(n, sizeof(uint32_t));
    for (size_t i = 0; i < a->n; i++) {
        uint64_t carry = 0;
        for (size_t k = 0; k < b->n; k++) {
            uint64_t t = (uint64_t)a->v[i] * b->v[k] + out[i + k] + carry;
            out[i + k] = (uint32_t)t;
            carry = t >> 32;
        }
        size_t k = i + b->n;
        while (carry) {
            uint64_t t = (uint64_t)out[k] + carry;
            out[k] = (uint32_t)t;
            carry = t >> 32;
            k++;
        }
    }
    free(r->v);
    r->v = out; r->n = n; r->cap = n;
    bn_trim(r);
}
/* decimal string of x into buf (cap bytes); returns needed length or -1 */
static long bn_to_dec(const bn *x, char *buf, size_t cap)
{
    bn t; bn_init(&t); bn_copy(&t, x);
    size_t maxd = t.n * 10 + 2;
    char *tmp = (char *)malloc(maxd);
    size_t k = 0;
    if (t.n == 0) tmp[k++] = '0';
    while (t.n) {
        uint64_t rem = 0;
        for (size_t i = t.n; i-- > 0;) {
            uint64_t cur = (rem << 32) | t.v[i];
            t.v[i] = (uint32_t)(cur / 10);
            rem = cur % 10;
        }
        bn_trim(&t);
        tmp[k++] = (char)('0' + rem);
    }
    long need = (long)k;
    if (buf && cap > k) {
        for (size_t i = 0; i < k; i++) buf[i] = tmp[k - 1 - i];
        buf[k] = 0;
    }
    free(tmp);
    bn_free(&t);
    return need;
}

/*
 * Big-integer mode: eps_d = (x0 + y0 sqrt d)/2 exactly.
 * Writes x0, y0 in decimal (if buffers are large enough), the norm sign
 * (+1 / -1 from x0^2 - d y0^2 = +-4; 0 if the norm check fails) and the
 * period.  Returns the Eisenstein flag (y0 even), or -1 on error.
 */
int orc_unit_bigint(uint64_t d, char *x0_dec, char *y0_dec, size_t cap,
                    int *norm_sign, uint64_t *period, uint64_t *y0_bits)
{
    if (d % 8 != 5 || d >= ((uint64_t)1 << 62)) return -1;
    const uint64_t s = orc_isqrt(d);
    uint64_t P = 1, Q = 2;
    bn A2, A1, B2, B1, A, B;
    bn_init(&A2); bn_init(&A1); bn_init(&B2); bn_init(&B1); bn_init(&A); bn_init(&B);
    bn_set_u64(&A2, 0); bn_set_u64(&A1, 1); bn_set_u64(&B2, 1); bn_set_u64(&B1, 0);
    bn zero; bn_init(&zero); bn_set_u64(&zero, 0);
    uint64_t j = 0;
    const int mut = g_mutation;
    int rc = 0;
    for (;;) {
        uint64_t q = (P + s) / Q;
        if (q >> 32) { rc = -1; break; }
        bn_mul_small_add(&A, &A1, (uint32_t)q, mut == 1 ? &zero : &A2);
        bn_mul_small_add(&B, &B1, (uint32_t)q, mut == 1 ? &zero : &B2);
        uint64_t Pn = q * Q - P;
        uint64_t sq = Pn * Pn;
        if (sq >= d || (d - sq) % Q != 0) { rc = -1; break; }
        uint64_t Qn = (d - sq) / Q;
        bn_copy(&A2, &A1); bn_copy(&A1, &A);
        bn_copy(&B2, &B1); bn_copy(&B1, &B);
        P = Pn; Q = Qn;
        j++;
        if (Q == 2) break;
        if (j > ORC_MAX_STEPS) { rc = -1; break; }
    }
    if (rc == 0) {
        /* x0 = 2 A_{l-1} - B_{l-1}, y0 = B_{l-1} */
        bn x0, y0, twoA, x2, y2, dd, dy2;
        bn_init(&x0); bn_init(&y0); bn_init(&twoA); bn_init(&x2); bn_init(&y2);
        bn_init(&dd); bn_init(&dy2);
        bn_add(&twoA, &A1, &A1);
        if (mut == 2) {
            bn_add(&x0, &twoA, &B1);
        } else if (bn_cmp(&twoA, &B1) >= 0) {
            bn_sub(&x0, &twoA, &B1);
        } else {
            /* cannot happen for a unit > 1; report as an error */
            rc = -1;
        }
        if (rc == 0) {
            bn_copy(&y0, &B1);
            bn_mul(&x2, &x0, &x0);
            bn_mul(&y2, &y0, &y0);
            bn_set_u64(&dd, d);
            bn_mul(&dy2, &dd, &y2);
            bn four; bn_init(&four); bn_set_u64(&four, 4);
            bn t; bn_init(&t);
            int sign = 0;
            if (bn_cmp(&x2, &dy2) >= 0) {
                bn_sub(&t, &x2, &dy2);
                if (bn_cmp(&t, &four) == 0) sign = +1;
            } else {
                bn_sub(&t, &dy2, &x2);
                if (bn_cmp(&t, &four) == 0) sign = -1;
            }
            if (norm_sign) *norm_sign = sign;
            if (period) *period = j;
            if (y0_bits) {
                size_t bitsz = 0;
                if (y0.n) {
                    uint32_t top = y0.v[y0.n - 1];
                    bitsz = (y0.n - 1) * 32;
                    while (top) { bitsz++; top >>= 1; }
                }
                *y0_bits = bitsz;
            }
            if (x0_dec) bn_to_dec(&x0, x0_dec, cap);
            if (y0_dec) bn_to_dec(&y0, y0_dec, cap);
            unsigned y0low = y0.n ? (y0.v[0] & 1) : 0;
            unsigned x0low = x0.n ? (x0.v[0] & 1) : 0;
            if (mut == 4) rc = (A1.n ? (A1.v[0] & 1) : 0) == 0;
            else rc = (y0low == 0 && x0low == 0) ? 1 : 0;
            bn_free(&four); bn_free(&t);
        }
        bn_free(&x0); bn_free(&y0); bn_free(&twoA); bn_free(&x2); bn_free(&y2);
        bn_free(&dd); bn_free(&dy2);
    }
    bn_free(&A2); bn_free(&A1); bn_free(&B2); bn_free(&B1); bn_free(&A); bn_free(&B);
    bn_free(&zero);
    return rc;
}

/* ------------------------------------------------------------------ */
/* Brute-force Pell search (Lemma 1.1 (2)).                            */
/* ------------------------------------------------------------------ */
/*
 * Least y in [1, ymax] such that d y^2 + 4 or d y^2 - 4 is a perfect square.
 * Returns y (0 if there is none up to ymax); *x_out gets the matching x and
 * *sign gets +1 (x^2 - d y^2 = 4) or -1 (= -4).  d y^2 must fit in 64 bits.
 */
uint64_t orc_pell_least_y(uint64_t d, uint64_t ymax, uint64_t *x_out, int *sign)
{
    for (uint64_t y = 1; y <= ymax; y++) {
        u128 t = (u128)d * y * y;
        if (t + 4 >= ((u128)1 << 64)) return 0;
        uint64_t tt = (uint64_t)t;
        uint64_t r = orc_isqrt(tt - 4);
        if (r * r == tt - 4) { if (x_out) *x_out = r; if (sign) *sign = -1; return y; }
        r = orc_isqrt(tt + 4);
        if (r * r == tt + 4) { if (x_out) *x_out = r; if (sign) *sign = +1; return y; }
    }
    return 0;
}

/* ------------------------------------------------------------------ */
/* Narrow class number by cycles of reduced indefinite forms.          */
/* ------------------------------------------------------------------ */
static int64_t gcd_i64(int64_t a, int64_t b)
{
    if (a < 0) a = -a;
    if (b < 0) b = -b;
    while (b) { int64_t t = a % b; a = b; b = t; }
    return a;
}

typedef struct { int64_t a, b, c; } form_t;

static int form_cmp(const void *x, const void *y)
{
    const form_t *f = (const form_t *)x, *g = (const form_t *)y;
    if (f->a != g->a) return f->a < g->a ? -1 : 1;
    if (f->b != g->b) return f->b < g->b ? -1 : 1;
    return 0;
}

/* (a,b,c) with b^2 - 4ac = D is reduced iff 0 < b < sqrt D and
 * sqrt D - b < 2|a| < sqrt D + b. */
static int form_is_reduced(int64_t a, int64_t b, int64_t D)
{
    if (b <= 0 || b * b >= D) return 0;
    int64_t A2 = 2 * (a < 0 ? -a : a);
    int64_t lo = A2 + b;  /* A2 > sqrt D - b  <=>  (A2 + b)^2 > D */
    if (lo * lo <= D) return 0;
    int64_t hi = A2 - b;  /* A2 < sqrt D + b  <=>  A2 - b < sqrt D */
    if (hi > 0 && hi * hi >= D) return 0;
    return 1;
}

/*
 * h+(D) for a positive non-square discriminant D = 0, 1 (mod 4): the number of
 * proper equivalence classes of primitive forms of discriminant D, counted as
 * the number of cycles of reduced forms under
 *   rho(a, b, c) = (c, b', (b'^2 - D)/(4c)),
 * b' = -b (mod 2|c|), sqrt D - 2|c| < b' < sqrt D
 * (rho composes the proper transformations (x,y) -> (-y, x) and a shear).
 * Returns -1 on error.
 */
int64_t orc_narrow_class_number(int64_t D)
{
    if (D <= 0 || (D % 4 != 0 && D % 4 != 1)) return -1;
    int64_t r = (int64_t)orc_isqrt((uint64_t)D);
    if (r * r == D) return -1;
    size_t cap = 1024, n = 0;
    form_t *F = (form_t *)malloc(cap * sizeof(form_t));
    for (int64_t b = 1; b <= r; b++) {
        if ((b - D) % 2 != 0) continue;
        int64_t m = (D - b * b) / 4; /* = -ac > 0 */
        for (int64_t a0 = 1; a0 <= m; a0++) {
            if (m % a0 != 0) continue;
            for (int sg = -1; sg <= 1; sg += 2) {
                int64_t a = sg * a0;
                int64_t c = -m / a;
                if (!form_is_reduced(a, b, D)) continue;
                if (gcd_i64(gcd_i64(a, b), c) != 1) continue;
                if (n == cap) { cap *= 2; F = (form_t *)realloc(F, cap * sizeof(form_t)); }
                F[n].a = a; F[n].b = b; F[n].c = c; n++;
            }
        }
    }
    qsort(F, n, sizeof(form_t), form_cmp);
    uint8_t *seen = (uint8_t *)calloc(n ? n : 1, 1);
    int64_t cycles = 0;
    for (size_t i = 0; i < n; i++) {
        if (seen[i]) continue;
        cycles++;
        form_t f = F[i];
        size_t guard = 0;
        for (;;) {
            form_t key = f;
            form_t *hit = (form_t *)bsearch(&key, F, n, sizeof(form_t), form_cmp);
            if (!hit) { cycles = -1; goto done; }
            size_t idx = (size_t)(hit - F);
            if (seen[idx]) break;
            seen[idx] = 1;
            int64_t c = f.c, ac = c < 0 ? -c : c;
            int64_t t = (r + f.b) % (2 * ac);
            if (t < 0) t += 2 * ac;
            int64_t bn_ = r - t; /* = -b mod 2|c|, largest below sqrt D */
            int64_t num = bn_ * bn_ - D;
            if (num % (4 * c) != 0) { cycles = -1; goto done; }
            form_t g; g.a = c; g.b = bn_; g.c = num / (4 * c);
            f = g;
            if (++guard > n + 1) { cycles = -1; goto done; }
        }
    }
done:
    free(F);
    free(seen);
    return cycles;
}

/* ------------------------------------------------------------------ */
/* Range classification (threads split the candidates dynamically).    */
/* ------------------------------------------------------------------ */
typedef struct {
    uint64_t d0, n;
    const uint8_t *sq;
    uint8_t *eis_bytes; /* one byte per candidate, written by one thread each */
    uint64_t next;      /* shared chunk counter */
    uint64_t steps;     /* total rho steps */
    int err;
    pthread_mutex_t mu;
} job_t;

#define ORC_CHUNK 64

static void *worker(void *arg)
{
    job_t *J = (job_t *)arg;
    uint64_t local_steps = 0;
    int local_err = 0;
    for (;;) {
        uint64_t i0 = __atomic_fetch_add(&J->next, ORC_CHUNK, __ATOMIC_RELAXED);
        if (i0 >= J->n) break;
        uint64_t i1 = i0 + ORC_CHUNK < J->n ? i0 + ORC_CHUNK : J->n;
        for (uint64_t i = i0; i < i1; i++) {
            if (!((J->sq[i / 8] >> (i % 8)) & 1)) { J->eis_bytes[i] = 0; continue; }
            uint64_t l = 0;
            int S = 0;
            int f = orc_walk_mod2(J->d0 + 8 * i, &l, &S);
            if (f < 0) { local_err = 1; f = 0; }
            J->eis_bytes[i] = (uint8_t)f;
            local_steps += l;
        }
    }
    pthread_mutex_lock(&J->mu);
    J->steps += local_steps;
    if (local_err) J->err = 1;
    pthread_mutex_unlock(&J->mu);
    return NULL;
}

/*
 * Classify every candidate d = d0 + 8 i in [a, b).  Bitmaps use the same
 * layout as orc_sqfree_range; either may be NULL.  nthreads <= 0 uses 1.
 * *total_steps (optional) gets the number of rho steps walked (full periods).
 * Returns 0 on success, -1 on error.
 */
int orc_classify_range(uint64_t a, uint64_t b, uint8_t *sq_bits, uint8_t *eis_bits,
                       size_t nbytes, uint64_t *n_sq, uint64_t *n_eis, int nthreads,
                       uint64_t *total_steps)
{
    uint64_t n = orc_num_candidates(a, b);
    size_t need = (size_t)((n + 7) / 8);
    if ((sq_bits || eis_bits) && nbytes < need) return -1;
    uint8_t *sq = (uint8_t *)calloc(need ? need : 1, 1);
    int64_t nsq = orc_sqfree_range(a, b, sq, need ? need : 1);
    if (nsq < 0) { free(sq); return -1; }
    uint8_t *eb = (uint8_t *)calloc(n ? n : 1, 1);
    job_t J;
    J.d0 = orc_first_candidate(a); J.n = n; J.sq = sq; J.eis_bytes = eb;
    J.next = 0; J.steps = 0; J.err = 0;
    pthread_mutex_init(&J.mu, NULL);
    if (nthreads <= 0) nthreads = 1;
    pthread_t *th = (pthread_t *)malloc(sizeof(pthread_t) * (size_t)nthreads);
    for (int t = 0; t < nthreads; t++) pthread_create(&th[t], NULL, worker, &J);
    for (int t = 0; t < nthreads; t++) pthread_join(th[t], NULL);
    free(th);
    pthread_mutex_destroy(&J.mu);
    uint64_t ne = 0;
    for (uint64_t i = 0; i < n; i++) ne += eb[i];
    if (sq_bits) { memset(sq_bits, 0, nbytes); memcpy(sq_bits, sq, need); }
    if (eis_bits) {
        memset(eis_bits, 0, nbytes);
        for (uint64_t i = 0; i < n; i++)
            if (eb[i]) eis_bits[i / 8] |= (uint8_t)(1u << (i % 8));
    }
    if (n_sq) *n_sq = (uint64_t)nsq;
    if (n_eis) *n_eis = ne;
    if (total_steps) *total_steps = J.steps;
    int err = J.err;
    free(sq);
    free(eb);
    return err ? -1 : 0;
}

/*
 * Classify an explicit list of d values (no squarefree test; the caller
 * passes members of D).  flags[i] = 1 if d[i] is Eisenstein.  Used to time
 * and check bounded samples of large ranges.  Returns 0 or -1.
 */
typedef struct {
    const uint64_t *d;
    uint8_t *flags;
    uint64_t n, next, steps;
    int err;
    pthread_mutex_t mu;
} listjob_t;

static void *list_worker(void *arg)
{
    listjob_t *J = (listjob_t *)arg;
    uint64_t local_steps = 0;
    int local_err = 0;
    for (;;) {
        uint64_t i = __atomic_fetch_add(&J->next, 1, __ATOMIC_RELAXED);
        if (i >= J->n) break;
        uint64_t l = 0;
        int S = 0;
        int f = orc_walk_mod2(J->d[i], &l, &S);
        if (f < 0) { local_err = 1; f = 0; }
        J->flags[i] = (uint8_t)f;
        local_steps += l;
    }
    pthread_mutex_lock(&J->mu);
    J->steps += local_steps;
    if (local_err) J->err = 1;
    pthread_mutex_unlock(&J->mu);
    return NULL;
}

int orc_classify_list(const uint64_t *d, uint64_t n, uint8_t *flags, int nthreads,
                      uint64_t *total_steps)
{
    listjob_t J;
    J.d = d; J.flags = flags; J.n = n; J.next = 0; J.steps = 0; J.err = 0;
    pthread_mutex_init(&J.mu, NULL);
    if (nthreads <= 0) nthreads = 1;
    pthread_t *th = (pthread_t *)malloc(sizeof(pthread_t) * (size_t)nthreads);
    for (int t = 0; t < nthreads; t++) pthread_create(&th[t], NULL, list_worker, &J);
    for (int t = 0; t < nthreads; t++) pthread_join(th[t], NULL);
    free(th);
    pthread_mutex_destroy(&J.mu);
    if (total_steps) *total_steps = J.steps;
    return J.err ? -1 : 0;
}
