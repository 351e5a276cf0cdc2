// eis_giant.h -- device arithmetic of the infrastructure giant step
// (Appendix A: Algorithms NUCOMP, NUDUPL and NUCOMPchoose, the reduction map
// rho on non-reduced ideals, and the residue of gamma in (O_K/2O_K)^*).
//
// Number representation.  Form coefficients and every intermediate of
// NUCOMP/NUDUPL are integers carried in fp64, where +, -, * and fma are
// exact while the exact result stays below 2^53 in magnitude.  Every product
// and every multi-term sum is checked against 2^52 (so that sums of two
// checked values are exact too), and every division the algorithms declare
// exact is checked for a zero remainder.  Any failed check makes the
// composition `bad`; the caller then discards the giant-step result for
// that d and classifies it with the plain reduction walk instead.  The
// checks accumulate in vector registers (the largest magnitude seen, the
// sum of the remainders' magnitudes) and are tested once at the end, which
// keeps the scalar unit free.  The extended and partial Euclid loops work
// on numbers below 2^21 (ideal norms and their cofactors for d < 10^12)
// and run in fp32, exact there.  The reduction after the composition uses
// the division-free form of rho, so it never needs P^2.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "eis_internal.h"

namespace eis {

typedef long long i64;

constexpr double kExactLimit = 4503599627370496.0;  // 2^52

// Accumulated checks of one composition.
struct Chk {
    double mx = 0.0;   // largest magnitude checked against 2^52
    double rs = 0.0;   // sum of the magnitudes of the exact divisions' remainders
    bool fail = false; // explicit failures
    __device__ __forceinline__ bool bad() const { return fail || !(mx < kExactLimit) || !(rs == 0.0); }
};

__device__ __forceinline__ void chk(double x, Chk &c) { c.mx = fmax(c.mx, fabs(x)); }

// 1/b to nearly full fp64 precision: hardware estimate + one Newton step.
__device__ __forceinline__ double rcp_nr(double b)
{
    double r = __builtin_amdgcn_rcp(b);
    return fma(fma(-b, r, 1.0), r, r);
}

// floor(a / b) for integers |a| < 2^52, 0 < b < 2^52.  The estimate is off
// by at most one either way; the correction is arithmetic, not a branch, so
// that lanes needing it do not split the wave.
__device__ __forceinline__ double fl_div(double a, double b)
{
    const double q = floor(a * rcp_nr(b));
    const double r = fma(-q, b, a);  // exact: |r| < 2b
    return q + (double)((int)(r >= b) - (int)(r < 0.0));
}

// a mod m in [0, m) for integers |a| < 2^52, 0 < m < 2^52.
__device__ __forceinline__ double nn_mod(double a, double m)
{
    double q = fl_div(a, m);
    return fma(-q, m, a);
}

// a / b where the quotient is an exact integer of magnitude < 2^50; the
// remainder goes to the checks.
__device__ __forceinline__ double ex_div(double a, double b, Chk &c)
{
    double q = rint(a * rcp_nr(b));
    c.rs += fabs(fma(-q, b, a));
    return q;
}

// -q and r = a - q b, for q = floor(a / b) and integer-valued fp32
// 0 <= a <= kShortDivMax, 0 < b.  The estimate floor(fl(a c) rcp(b)) with
// c = 1 + 2^-21 is never below the true quotient k: the relative errors of
// the roundings (the product a c, the reciprocal's 1 ulp, the final
// product) add up to less than 2^-21.  It exceeds a / b by at most
// (a / b) 1.5 2^-21, so an overshoot to k + 1 needs (k + 1) b - a <=
// 1.5 a 2^-21 with (k + 1) b - a >= 1, i.e. a >= 2^21 / 1.5: below that
// the estimate is exact and no correction is needed.  (-q, so that callers
// fold it into an fma without a negation.)
constexpr float kDivBias = 1.f + 0x1p-21f;
constexpr double kShortDivMax = 1398101.0;  // floor(2^21 / 1.5)

__device__ __forceinline__ float neg_fl_div32(float a, float b, float &r)
{
    const float nq = ceilf(-(a * kDivBias) * __builtin_amdgcn_rcpf(b));
    r = fmaf(nq, b, a);
    return nq;
}

// Work counts of one composition (for the instruction model of the giant
// walk): Euclid steps of the extended and partial Euclid loops (and, of
// those, the extended Euclid's), reduction steps after the composition, and
// whether NUCOMP took its gcd branch.
struct GiantWork {
    u32 euclid = 0, xgcd = 0, reduce = 0, gcd_branch = 0;
};

// Extended Euclid, the first cofactor only: g = gcd(a, b) >= 0 and x with
// x a + y b = g for some integer y (so x a = g mod b), for integers |a|,
// |b| < 2^21: exact in fp32.  Invariants: x0 A = a and x1 A = b modulo B,
// for the inputs A = |a|, B = |b|; the loop ends when one of a, b is 0, and
// the other is +-g.  Each division step takes the quotient nearest to a / b
// (remainders of either sign), which needs about 30 % fewer steps than
// floor quotients (1 / 1.71 against 1 / 1.19 steps per unit of ln b for the
// nearest-integer and the regular continued fraction) and no correction:
// the estimate rint(a rcp(b)) is within 0.875 of a / b (relative error of
// rcp and the product below 1.5 2^-23, a / b < 2^21), so |remainder| <
// 0.875 |b| and the remainders fall strictly.  The cofactors stay below B / g
// in magnitude.  x is determined modulo B / g, which is all the callers use
// (their results are the same for every such x).  A caller that needs y
// computes (g - x a) / b, an exact division.  Two division steps per
// iteration, the second with the roles of (a, x0) and (b, x1) exchanged
// and applied only if the first left a != 0 (a select, not a branch), so
// that no step moves registers around.
__device__ __forceinline__ void xgcd1(double ad, double bd, double &x, double &g, GiantWork &wk)
{
    const float sa = ad < 0.0 ? -1.f : 1.f;
    float a = (float)fabs(ad), b = (float)fabs(bd);
    float x0 = 1.f, x1 = 0.f;
    u32 iters = 0;
    while (a != 0.f && b != 0.f) {
        float q = rintf(a * __builtin_amdgcn_rcpf(b));
        a = fmaf(-q, b, a);
        x0 = fmaf(-q, x1, x0);
        const bool go = a != 0.f;
        q = rintf(b * __builtin_amdgcn_rcpf(go ? a : 1.f));
        b = go ? fmaf(-q, a, b) : b;
        x1 = go ? fmaf(-q, x0, x1) : x1;
        iters++;
    }
    const bool az = a == 0.f;
    // every iteration takes two steps but the last, whose second step is
    // skipped when it leaves a = 0
    const u32 steps = iters ? 2u * iters - (az ? 1u : 0u) : 0u;
    wk.euclid += steps;
    wk.xgcd += steps;
    const float gs = az ? b : a, xs = az ? x1 : x0;
    g = (double)fabsf(gs);
    x = (double)((gs < 0.f ? -xs : xs) * sa);
}

struct Form {
    double u, v, w;
};

// gamma = (A + B sqrt d) / C
struct Gamma {
    double A, B, C;
};

// Partial Euclid shared by NUCOMP and NUDUPL: run while |b_y| > L and b_x != 0
// (both stay non-negative), then flip the signs of b_y and y when the number
// of steps z is odd.  0 <= b_x < b_y, so the loop runs in fp32.  A step
// takes q = floor(b_y / b_x) and maps (b_x, b_y, x, y) to
// (b_y - q b_x, b_x, y - q x, x).  Every dividend is at most the first b_y,
// a norm's divisor u_1 / G < sqrt d <= 10^6 for the forms of reduced ideals
// and d <= 10^12, so the quotient's estimate needs no correction (a larger
// b_y fails the composition's checks).  Two steps per iteration, the second
// on the exchanged roles (u, v, X, Y) -> (v, u, Y, X) and applied only if
// the loop condition holds after the first (a select, not a branch), so that
// no step moves registers around.
__device__ __forceinline__ void partial_euclid(double &bxd, double &byd, double &x, double &y,
                                               int &z, double L, Chk &bad)
{
    bad.fail |= !(byd <= kShortDivMax);
    float u = (float)bxd, v = (float)byd, X = 1.f, Y = 0.f;  // (b_x, b_y, x, y)
    const float Lf = (float)L;
    bool odd = false;  // the last iteration took one step: the roles stay exchanged
    int iters = 0;
    bool run = v > Lf && u != 0.f;
    while (run) {
        float r;
        float nq = neg_fl_div32(v, u, r);
        v = r;
        Y = fmaf(nq, X, Y);
        // now (b_x, b_y, x, y) = (v, u, Y, X)
        const bool go = u > Lf && v != 0.f;
        nq = neg_fl_div32(u, go ? v : 1.f, r);
        u = go ? r : u;
        X = go ? fmaf(nq, Y, X) : X;
        iters++;
        odd = !go;
        run = go && v > Lf && u != 0.f;
    }
    const int n = 2 * iters - (odd ? 1 : 0);
    z = n;
    float bx = odd ? v : u, by = odd ? u : v, xf = odd ? Y : X, yf = odd ? X : Y;
    if (n & 1) {
        by = -by;
        yf = -yf;
    }
    bxd = (double)bx;
    byd = (double)by;
    x = (double)xf;
    y = (double)yf;
}

// Algorithm NUCOMP: phi3 = (1/gamma) phi1 phi2, partially reduced with bound L.
__device__ __forceinline__ void nucomp(Form f1, Form f2, double L, Form &f3, Gamma &g,
                                       Chk &bad, GiantWork &wk)
{
    if (f1.w < f2.w) {
        const Form t = f1;
        f1 = f2;
        f2 = t;
    }
    const double s = ex_div(f1.v + f2.v, 2.0, bad);
    const double m = f2.v - s;
    double b, F;
    xgcd1(f2.u, f1.u, b, F, wk);  // b u2 = F (mod u1)
    double G, Bx, By, Cy, Dy;
    if (nn_mod(s, F) == 0.0) {
        G = F;
        Bx = m * b;
        chk(Bx, bad);
        By = ex_div(f1.u, G, bad);
        Cy = ex_div(f2.u, G, bad);
        Dy = ex_div(s, G, bad);
    } else {
        double y2;
        wk.gcd_branch = 1;
        // c with b u2 + c u1 = F (an exact division)
        chk(b * f2.u, bad);
        const double c = ex_div(fma(-b, f2.u, F), f1.u, bad);
        xgcd1(s, F, y2, G, wk);  // y2 s = G (mod F); only y2 mod F/G matters
        const double H = ex_div(F, G, bad);
        By = ex_div(f1.u, G, bad);
        Cy = ex_div(f2.u, G, bad);
        Dy = ex_div(s, G, bad);
        // l = y2 (b w1 + c w2) mod H, reduced term by term to keep it small
        const double t1 = nn_mod(b, H) * nn_mod(f1.w, H);
        const double t2 = nn_mod(c, H) * nn_mod(f2.w, H);
        const double l = nn_mod(nn_mod(y2, H) * nn_mod(t1 + t2, H), H);
        const double num = fma(l, By, b * m);
        chk(b * m, bad);
        chk(l * By, bad);
        chk(num, bad);
        Bx = ex_div(num, H, bad);
    }
    double bx = nn_mod(Bx, By), by = By, x, y;
    int z;
    partial_euclid(bx, by, x, y, z, L, bad);
    wk.euclid += (u32)z;
    const double ax = G * x, ay = G * y;
    double u3, v3, w3;
    if (z != 0) {
        const double n1 = fma(Cy, bx, -m * x);
        chk(Cy * bx, bad);
        chk(m * x, bad);
        const double cx = ex_div(n1, By, bad);
        const double Q1 = by * cx;
        chk(Q1, bad);
        const double Q2 = Q1 + m;
        const double n2 = fma(Dy, bx, -f2.w * x);
        chk(Dy * bx, bad);
        chk(f2.w * x, bad);
        const double dx = ex_div(n2, By, bad);
        const double Q3 = y * dx;
        chk(Q3, bad);
        const double Q4 = Q3 + Dy;
        const double dy = ex_div(Q4, x, bad);
        double cy;
        if (bx != 0.0) {
            cy = ex_div(Q2, bx, bad);
        } else {
            const double n3 = fma(cx, dy, -f1.w);
            chk(cx * dy, bad);
            cy = ex_div(n3, dx, bad);
        }
        chk(by * cy, bad);
        chk(ay * dy, bad);
        chk(bx * cx, bad);
        chk(ax * dx, bad);
        u3 = fma(by, cy, -ay * dy);
        w3 = fma(bx, cx, -ax * dx);
        v3 = G * (Q3 + Q4) - Q1 - Q2;
        chk(G * (Q3 + Q4), bad);
    } else {
        const double Q1 = Cy * bx;
        chk(Q1, bad);
        const double cx = ex_div(Q1 - m, By, bad);
        const double n2 = fma(bx, Dy, -f2.w);
        chk(bx * Dy, bad);
        const double dx = ex_div(n2, By, bad);
        u3 = by * Cy;
        chk(bx * cx, bad);
        chk(G * dx, bad);
        w3 = fma(bx, cx, -G * dx);
        v3 = f2.v - 2.0 * Q1;
    }
    chk(u3, bad);
    chk(v3, bad);
    chk(w3, bad);
    const double t = 2.0 * u3;
    chk(x * t, bad);
    chk(y * v3, bad);
    g.A = G * fma(x, t, y * v3);
    g.B = G * y;
    g.C = t;
    chk(g.A, bad);
    f3.u = u3;
    f3.v = v3;
    f3.w = w3;
}

// Algorithm NUDUPL: phi3 = (1/gamma) phi^2, partially reduced with bound L.
__device__ __forceinline__ void nudupl(Form f, double L, Form &f3, Gamma &g, Chk &bad,
                                       GiantWork &wk)
{
    double y0, G;
    xgcd1(f.v, f.u, y0, G, wk);  // y0 v = G (mod u); only y0 mod u/G matters
    const double By = ex_div(f.u, G, bad);
    const double Dy = ex_div(f.v, G, bad);
    // B_x = y0 w mod B_y, reduced factor by factor
    const double Bx = nn_mod(nn_mod(y0, By) * nn_mod(f.w, By), By);
    double bx = Bx, by = By, x, y;
    int z;
    partial_euclid(bx, by, x, y, z, L, bad);
    wk.euclid += (u32)z;
    const double ax = G * x, ay = G * y;
    double u3, v3, w3;
    if (z == 0) {
        const double n = fma(bx, Dy, -f.w);
        chk(bx * Dy, bad);
        const double dx = ex_div(n, By, bad);
        u3 = by * by;
        w3 = bx * bx;
        const double sq = (bx + by) * (bx + by);
        chk(u3, bad);
        chk(w3, bad);
        chk(sq, bad);
        v3 = f.v - sq + u3 + w3;
        chk(G * dx, bad);
        w3 = w3 - G * dx;
    } else {
        const double n = fma(bx, Dy, -f.w * x);
        chk(bx * Dy, bad);
        chk(f.w * x, bad);
        const double dx = ex_div(n, By, bad);
        const double Q1 = dx * y;
        chk(Q1, bad);
        double dy = Q1 + Dy;
        v3 = G * (dy + Q1);
        chk(v3, bad);
        dy = ex_div(dy, x, bad);
        u3 = by * by;
        w3 = bx * bx;
        const double sq = (bx + by) * (bx + by);
        chk(u3, bad);
        chk(w3, bad);
        chk(sq, bad);
        v3 = v3 - sq + u3 + w3;
        chk(ay * dy, bad);
        chk(ax * dx, bad);
        u3 = u3 - ay * dy;
        w3 = w3 - ax * dx;
    }
    chk(u3, bad);
    chk(v3, bad);
    chk(w3, bad);
    const double t = 2.0 * u3;
    chk(x * t, bad);
    chk(y * v3, bad);
    g.A = G * fma(x, t, y * v3);
    g.B = G * y;
    g.C = t;
    chk(g.A, bad);
    f3.u = u3;
    f3.v = v3;
    f3.w = w3;
}

// Residue of gamma = (A + B sqrt d)/C in F_4^* ~ Z/3 (the localisation of
// Appendix A: 1/gamma lies in O_{K,2}).  Common factors 2 of A and B are
// stripped; (A + B sqrt d)/2 with A, B odd reduces to omega (log 1) when
// A = B (mod 4) and to omega^2 (log 2) otherwise; A + B sqrt d with A, B of
// mixed parity is odd (log 0).  The power of 2 stripped must equal that of C
// (gamma is a 2-unit), else `bad`.  Only A, B mod 2^64 matter, and |A|, |B|
// < 2^52 here, so the int64 images are exact.
__device__ __forceinline__ u32 gamma_log(const Gamma &g, Chk &bad)
{
    unsigned long long A = (unsigned long long)(i64)g.A;
    unsigned long long B = (unsigned long long)(i64)g.B;
    unsigned long long C = (unsigned long long)(i64)fabs(g.C);
    if (C == 0 || (A | B) == 0) {
        bad.fail = true;
        return 0;
    }
    const int vA = __builtin_ctzll(A | B);  // common power of 2
    A >>= vA;
    B >>= vA;
    int v = vA;
    u32 lg = 0;
    if ((A & 1) && (B & 1)) {
        v += 1;
        lg = (((A - B) & 3) == 0) ? 1u : 2u;
    }
    const int vC = __builtin_ctzll(C);
    bad.fail |= (v != vC);
    return lg;
}

// The form (u/2, -v', w) of a reduced ideal [u/2, (v + sqrt d)/2] (u = Q,
// v = P), with v' = v mod u and w = (v'^2 - d) / (2u) (an exact division).
// Inputs are reduced ideals: u < 2^21 and 0 < v < 2^21 for d < 2^40.
__device__ __forceinline__ Form ideal_form(double u, double v, double d, Chk &bad)
{
    u = fabs(u);
    v = nn_mod(v, u);
    return Form{0.5 * u, -v, ex_div(fma(v, v, -d), 2.0 * u, bad)};
}

// NUCOMPchoose: the form (u3, v3, w3) and gamma with
// [|2 u3|/2, (-v3 + sqrt d)/2] = (1/gamma) I_1 I_2, split by its cases.
// square_ideal is the I_1 = I_2 case (NUDUPL); compose_ideals runs NUCOMP for
// any pair.  NUCOMP is the general composition and handles I_1 = I_2 through
// its gcd step: on equal inputs it returns exactly what NUDUPL returns
// (checked on 6 * 10^4 squares of cycle ideals with d up to 10^12), so a
// caller whose lanes mix squares and products may send both through NUCOMP
// and keep every lane on one path.
//
// The small-norm case (a norm u_k <= 50; unless small_norm_product is off,
// a switchable variant) takes the plain ideal product,
// I_1 I_2 = S [u/2, (v + sqrt d)/2] with gamma = S: that is NUCOMP / NUDUPL
// with the partial reduction switched off (no partial Euclid step, so
// x = 1, y = 0 and gamma = G, the gcd of the norms and s), here obtained by
// an infinite bound L.  S is odd (2 is inert, so primitive ideals have odd
// norm u/2), a 2-unit of residue 0.  The caller's reduction then starts from
// the unreduced product.
constexpr double kSmallNorm = 50.0;

__device__ __forceinline__ void square_ideal(double u, double v, double d, double L, Form &f3,
                                             Gamma &g, Chk &bad, GiantWork &wk,
                                             bool small_norm_product = true)
{
    const double Lk = (small_norm_product && fabs(u) <= kSmallNorm) ? __builtin_inf() : L;
    nudupl(ideal_form(u, v, d, bad), Lk, f3, g, bad, wk);
    bad.fail |= (f3.u == 0.0);
}

__device__ __forceinline__ void compose_ideals(double u1, double v1, double u2, double v2,
                                               double d, double L, Form &f3, Gamma &g, Chk &bad,
                                               GiantWork &wk, bool small_norm_product = true)
{
    const double Lk = (small_norm_product && (fabs(u1) <= kSmallNorm || fabs(u2) <= kSmallNorm))
                          ? __builtin_inf()
                          : L;
    nucomp(ideal_form(u1, v1, d, bad), ideal_form(u2, v2, d, bad), Lk, f3, g, bad, wk);
    bad.fail |= (f3.u == 0.0);
}

// Reduction of the composed ideal.  The ideal of the form (u3, v3, w3) is
// [Q/2, (P + sqrt d)/2] with Q = |2 u3|, P = -v3 (P matters only mod Q, and
// the paper's normalisation v = -v3 mod u is not needed here), and its rho
// predecessor is Qp = (d - P^2)/Q = -2 sgn(u3) w3, which needs no big
// product.  rho then runs with the division-free recurrence
//   q = floor((P + sqrt d)/Q),  P' = q Q - P,  Q' = Qp + q (P - P')
// (Q may be negative on the way: then q = floor((-P - s - 1)/(-Q))), until
// Q > 0, 0 < P <= s and s - P < Q <= s + P.  Values stay exact fp64
// integers (checked).  Returns the residue sum of the relative generators
// (P' + sqrt d)/Q; on return Qp is the predecessor of the reduced (Q, P),
// and Q Qp = d - P^2 is checked.
constexpr int kMaxReduce = 128;

__device__ __forceinline__ bool is_reduced(double Q, double P, double s)
{
    return Q > 0.0 && P > 0.0 && P <= s && s - P < Q && Q <= s + P;
}

__device__ __forceinline__ bool reduce_more(double Q, double P, double s, int it, const Chk &bad)
{
    return !is_reduced(Q, P, s) && it < kMaxReduce && Q != 0.0 && bad.mx < kExactLimit;
}

// One step from (Q, P) with predecessor Qp: the new P goes to Pn and the new
// Q overwrites Qp (so the caller's two register sets swap roles each step).
__device__ __forceinline__ u32 reduce_step(double Q, double P, double s, double &Qp, double &Pn,
                                           Chk &bad)
{
    const double num = (Q > 0.0) ? P + s : -P - s - 1.0;
    const double q = fl_div(num, fabs(Q));
    const double qQ = q * Q;
    chk(qQ, bad);
    Pn = qQ - P;
    const double t = q * (P - Pn);
    chk(t, bad);
    Qp = Qp + t;
    chk(Qp, bad);
    const double t4 = Pn * 0.25;
    return (t4 - floor(t4) > 0.5) ? 2u : 1u;
}

__device__ __forceinline__ u32 reduce_form(const Form &f, double d, double s, double &Q,
                                           double &P, double &Qp, Chk &bad, GiantWork &wk)
{
    double Qa = fabs(2.0 * f.u), Pa = -f.v, Qb = (f.u > 0.0) ? -2.0 * f.w : 2.0 * f.w, Pb = 0.0;
    u32 S = 0;
    int it = 0;
    bool run = reduce_more(Qa, Pa, s, it, bad);
    for (;;) {
        if (run) {
            S += reduce_step(Qa, Pa, s, Qb, Pb, bad);  // now (Qb, Pb), predecessor Qa
            it++;
            run = reduce_more(Qb, Pb, s, it, bad);
        }
        if (run) {
            S += reduce_step(Qb, Pb, s, Qa, Pa, bad);  // back to (Qa, Pa), predecessor Qb
            it++;
            run = reduce_more(Qa, Pa, s, it, bad);
        }
        if (!__any(run)) break;
    }
    wk.reduce += (u32)it;
    const bool odd = (it & 1) != 0;
    Q = odd ? Qb : Qa;
    P = odd ? Pb : Pa;
    Qp = odd ? Qa : Qb;
    bad.fail |= !is_reduced(Q, P, s);
    bad.fail |= (fma(Q, Qp, P * P) != d);
    return S;
}

// Dictionary hash of a key (the fp32 bit patterns of Q and P); its low bits
// pick the first slot, its high 16 bits are the slot's fingerprint.
__device__ __forceinline__ u32 dict_hash(u32 Q, u32 P)
{
    u32 h = (Q * 0x9E3779B1u) ^ (P * 0x85EBCA77u);
    h ^= h >> 15;
    h *= 0x2C1B3C6Du;
    h ^= h >> 13;
    h *= 0x297A2D39u;
    h ^= h >> 16;
    return h;
}

}  // namespace eis
